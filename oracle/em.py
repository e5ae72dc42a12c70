"""Electromagnetics for the oracle: materials, Fresnel reflection, antenna
patterns and the polarised field transfer at a specular reflection.

Test infrastructure: see the package docstring.

The paper characterises a radio material by its relative permittivity eps_r
and conductivity sigma with mu_r = 1 (Sec. II) and transforms the polarised
field components at every interaction (Sec. II); the formulas are the textbook
ones, with these conventions:

* time dependence exp(+j w t); complex relative permittivity
  eta = eps_r - j sigma / (eps0 w); sigma = +inf is a perfect conductor with
  r_perp = -1 and r_par = +1 exactly.
* Fresnel:  s = sqrt(eta - sin^2 theta) (principal branch),
  r_perp = (cos - s)/(cos + s),  r_par = (eta cos - s)/(eta cos + s).
* Reflection of a unit direction d on a plane with normal n (n . d < 0 after
  flipping): d' = d - 2 (d.n) n.  Bases e_perp = d x n / |d x n| (any unit
  vector orthogonal to d at normal incidence), e_par_i = e_perp x d,
  e_par_r = e_perp x d'.  Field update on the complex Cartesian vector:
  E' = r_perp (E . e_perp) e_perp + r_par (E . e_par_i) e_par_r.
* Spherical unit vectors theta_hat = (cos t cos p, cos t sin p, -sin t),
  phi_hat = (-sin p, cos p, 0); at the poles phi = 0.
* Antenna orientation R = Rz(yaw) Ry(pitch) Rx(roll) (3GPP TR 38.901
  Sec. 7.1); a global direction d is seen locally as R^T d; the radiated
  field is F = R (C_theta theta_hat' + C_phi phi_hat').  Positive pitch tilts
  the boresight (+x) towards -z.
* Patterns (vertical polarisation, C_phi = 0): isotropic C_theta = 1;
  TR 38.901 Table 7.3-1 element: A_V = -min(12((theta-90)/65)^2, 30),
  A_H = -min(12(phi/65)^2, 30), A = -min(-(A_V + A_H), 30) dB (angles in
  degrees), gain 8 dBi + A, C_theta = 10^(G/20).
"""
from __future__ import annotations

import numpy as np

from .consts import EPS0

PATTERN_ISO = 0
PATTERN_TR38901 = 1
PATTERN_DIPOLE = 2
# single-port polarisation: C_theta = g cos(zeta), C_phi = g sin(zeta)
# (the polarisation model 2 of 3GPP TR 38.901 Sec. 7.3.2)
POL_ANGLE = {0: 0.0, 1: np.pi / 2, 2: np.pi / 4, 3: -np.pi / 4}   # V, H, +45 deg, -45 deg


def eta(eps_r, sigma, freq_hz):
    """Complex relative permittivity (array-friendly); inf sigma gives -1j*inf."""
    eps_r = np.asarray(eps_r, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    with np.errstate(invalid="ignore"):
        return eps_r - 1j * sigma / (EPS0 * 2.0 * np.pi * freq_hz)


def fresnel(eta_c, cos_i, pec=None):
    """(r_perp, r_par) for incidence cosine cos_i in (0, 1]."""
    eta_c = np.asarray(eta_c, dtype=np.complex128)
    cos_i = np.asarray(cos_i, dtype=np.float64)
    sin2 = 1.0 - cos_i * cos_i
    with np.errstate(invalid="ignore", divide="ignore"):
        s = np.sqrt(eta_c - sin2)
        r_perp = (cos_i - s) / (cos_i + s)
        r_par = (eta_c * cos_i - s) / (eta_c * cos_i + s)
    if pec is None:
        pec = ~np.isfinite(eta_c)
    pec = np.broadcast_to(pec, np.broadcast(r_perp, r_par).shape)
    r_perp = np.where(pec, -1.0 + 0j, r_perp)
    r_par = np.where(pec, 1.0 + 0j, r_par)
    return r_perp, r_par


def rot_matrix(yaw, pitch, roll):
    cy, sy = np.cos(yaw), np.sin(yaw)
    cp, sp = np.cos(pitch), np.sin(pitch)
    cr, sr = np.cos(roll), np.sin(roll)
    Rz = np.array([[cy, -sy, 0.0], [sy, cy, 0.0], [0.0, 0.0, 1.0]])
    Ry = np.array([[cp, 0.0, sp], [0.0, 1.0, 0.0], [-sp, 0.0, cp]])
    Rx = np.array([[1.0, 0.0, 0.0], [0.0, cr, -sr], [0.0, sr, cr]])
    return Rz @ Ry @ Rx


def theta_phi(d):
    d = np.asarray(d, dtype=np.float64)
    th = np.arccos(np.clip(d[..., 2], -1.0, 1.0))
    ph = np.arctan2(d[..., 1], d[..., 0])
    return th, ph


def theta_hat(th, ph):
    return np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)], axis=-1)


def phi_hat(ph):
    return np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)], axis=-1)


def amplitude(pid, th, ph):
    """Field amplitude g of a pattern for local angles (radians): isotropic 1;
    TR 38.901 Table 7.3-1 element; short dipole along the local z axis,
    sqrt(1.5) sin(theta) (directivity 1.5, i.e. 1.76 dBi)."""
    th = np.asarray(th, dtype=np.float64)
    ph = np.asarray(ph, dtype=np.float64)
    if pid == PATTERN_ISO:
        return np.ones_like(th)
    if pid == PATTERN_TR38901:
        tdeg = np.degrees(th)
        pdeg = np.degrees(ph)
        a_v = -np.minimum(12.0 * ((tdeg - 90.0) / 65.0) ** 2, 30.0)
        a_h = -np.minimum(12.0 * (pdeg / 65.0) ** 2, 30.0)
        a = -np.minimum(-(a_v + a_h), 30.0)
        return 10.0 ** ((8.0 + a) / 20.0)
    if pid == PATTERN_DIPOLE:
        return np.sqrt(1.5) * np.sin(th)
    raise ValueError("unknown pattern %r" % (pid,))


def pattern(pid, th, ph, pol=0):
    """(C_theta, C_phi) for local angles (radians) and a polarisation code."""
    g = amplitude(pid, th, ph)
    zeta = POL_ANGLE[int(pol)]
    return g * np.cos(zeta), g * np.sin(zeta)


def antenna_field(dev, d):
    """Radiated (or receive) field vector, global Cartesian, for global unit
    directions d (n, 3); dev has yaw, pitch, roll, pattern."""
    R = rot_matrix(dev.yaw, dev.pitch, dev.roll)
    dl = np.asarray(d, dtype=np.float64) @ R  # = (R^T d) per row
    th, ph = theta_phi(dl)
    ct, cp = pattern(dev.pattern, th, ph, getattr(dev, "pol", 0))
    f_local = ct[..., None] * theta_hat(th, ph) + cp[..., None] * phi_hat(ph)
    return f_local @ R.T


def reflect(d, n):
    """Specular reflection: returns (d', n_f, cos_i) with n_f facing the ray."""
    d = np.asarray(d, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    dn = np.einsum("...i,...i->...", d, n)
    n_f = np.where((dn > 0.0)[..., None], -n, n)
    cos_i = -np.einsum("...i,...i->...", d, n_f)
    d_r = d + 2.0 * cos_i[..., None] * n_f
    return d_r, n_f, cos_i


def perp_basis(d, n_f):
    """e_perp = d x n / |d x n|, or a unit vector orthogonal to d when d || n."""
    e = np.cross(d, n_f)
    nrm = np.linalg.norm(e, axis=-1)
    small = nrm < 1e-12
    if np.any(small):
        ds = d[small]
        # Gram-Schmidt of the axis least aligned with d
        ax = np.zeros_like(ds)
        ax[np.arange(ds.shape[0]), np.argmin(np.abs(ds), axis=-1)] = 1.0
        alt = ax - np.einsum("ij,ij->i", ax, ds)[:, None] * ds
        e[small] = alt
        nrm = np.where(small, np.linalg.norm(e, axis=-1), nrm)
    return e / nrm[..., None]


def transfer(E, d, d_r, n_f, r_perp, r_par):
    """Field after one reflection (complex Cartesian E, shape (n, 3))."""
    e_perp = perp_basis(d, n_f)
    e_par_i = np.cross(e_perp, d)
    e_par_r = np.cross(e_perp, d_r)
    a_perp = np.einsum("...i,...i->...", E, e_perp)
    a_par = np.einsum("...i,...i->...", E, e_par_i)
    return (np.asarray(r_perp)[..., None] * a_perp[..., None] * e_perp
            + np.asarray(r_par)[..., None] * a_par[..., None] * e_par_r)


def transfer_scattered(E, d, d_s, n_f, r_perp, r_par):
    """Field of a diffusely scattered ray leaving in direction d_s: the
    reflected components r_perp a_perp, r_par a_par of the incident field,
    carried by the transverse basis of d_s (e_perp' = d_s x n / |d_s x n|,
    e_par' = e_perp' x d_s).  For d_s the specular direction this is transfer()."""
    e_perp = perp_basis(d, n_f)
    e_par_i = np.cross(e_perp, d)
    s_perp = perp_basis(d_s, n_f)
    s_par = np.cross(s_perp, d_s)
    a_perp = np.einsum("...i,...i->...", E, e_perp)
    a_par = np.einsum("...i,...i->...", E, e_par_i)
    return (np.asarray(r_perp)[..., None] * a_perp[..., None] * s_perp
            + np.asarray(r_par)[..., None] * a_par[..., None] * s_par)


def wavelength(freq_hz):
    from .consts import C0
    return C0 / freq_hz
