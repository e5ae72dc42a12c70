"""Diffusely scattered paths (FP64).

Test infrastructure: see the package docstring.

Sec. II-B names diffuse reflection (scattering) among the interactions the ray
tracer computes, and Sec. II-A says scattering can be enabled when paths are
computed; the paper leaves the model to its documentation.  The model used
here is the Lambertian one of ``oracle.scatter`` (a scattering coefficient S
per material: the fraction S^2 of the reflected power is scattered diffusely,
1 - S^2 stays specular), turned into paths with the ray tubes of the
Fibonacci lattice:

* the lattice rays of the transmitter are traced with specular reflections,
  as for path candidates (closest hit, the last face skipped, t_min);
* hit k = 1..max_depth of lattice ray i, at the point h of face f (unit normal
  n facing the ray, incident direction d, ray length s from the transmitter),
  scatters towards every receiver R in front of the face ((R - h) . n > 0)
  whose open segment h -> R is unoccluded (face f skipped at its start, as
  for the segments of image paths);
* the ray stands for the solid angle 4 pi / N, so at distance s it lights the
  area s^2 (4 pi / N) / cos_i.  A Lambertian patch re-radiates the scattered
  power with the intensity pattern cos_s / pi; the 1/s^2 of the incident power
  density cancels against the lit area, and
      a = lambda / (4 pi) * S_f * w * sqrt((4 pi / N) cos_s / pi) / r_s
          * F_rx(-k) . E_s,
  with k = (R - h) / r_s, r_s = |R - h|, cos_s = k . n,
  E_s = em.transfer_scattered(E, d, k, n, r_perp, r_par) the reflected
  components of the ray's field E (F_tx(d_0) times the earlier reflection
  operators) carried by the transverse basis of k, and w the product of
  sqrt(1 - S^2) over the earlier reflections (their specular share; with
  scattering coefficients the specular paths of ``oracle.image`` carry the
  same factor per reflection);
* the carrier phase exp(-j 2 pi f tau) is not part of a, tau = (s + r_s)/c0,
  AoD = angles of d_0, AoA = angles of -k (global frame);
* T[i, j] = L c b_i(k) . E_s(u_j), L = s + r_s, c = a's real scalar factor
  S_f w sqrt(...) / r_s, u_j = (theta_hat(d_0), phi_hat(d_0)) carried like E,
  b_i = (theta_hat(k), phi_hat(k)); then, as for image paths,
  a = lambda / (4 pi L) sum_ij (F_rx(-k) . b_i) T[i, j] (F_tx(d_0) . u_j).

Sub-lattices (ray_begin, ray_stride) trace only their rays, each with the
weight 4 pi / N of the full lattice.  The paths of a receiver are ordered by
(lattice ray, depth).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import em, fib, native
from .consts import C0, OCC_EPS
from .geom import Geometry


@dataclass
class ScatPath:
    rx: int
    ray: int             # lattice index of the ray
    depth: int           # interactions: k - 1 specular reflections, then the scattering
    faces: tuple         # faces of the k hits, the scattering face last
    a: complex
    T: np.ndarray        # (2, 2) complex
    tau: float
    length: float
    aod: tuple
    aoa: tuple
    point: np.ndarray    # scattering point h


def _angles(d):
    th, ph = em.theta_phi(d)
    return float(th), float(ph)


def paths(scene, tx, rxs, params, S, geo=None, threads=None):
    """Scattered paths of one transmitter for every receiver: a list (per rx)
    of ScatPath sorted by (ray, depth).  ``params`` is an oracle.sbr.TraceParams
    (num_rays N, max_depth, tmin, ray_begin, ray_stride); ``S`` the scattering
    coefficient per material (taken in float32, as stored by the library)."""
    geo = geo or Geometry(scene)
    lam = C0 / geo.freq
    N = int(params.num_rays)
    S = np.asarray(S, dtype=np.float32).astype(np.float64)
    idx = fib.subset(N, params.ray_begin, params.ray_stride)
    n = idx.shape[0]
    d0 = fib.directions(N, idx)
    th0, ph0 = em.theta_phi(d0)
    U = np.stack([em.theta_hat(th0, ph0), em.phi_hat(ph0)], axis=1).astype(np.complex128)  # (n, 2, 3)
    Ftx = em.antenna_field(tx, d0)
    ftx = np.einsum("nij,nj->ni", U.real, Ftx)          # departure components (theta, phi)
    o = np.repeat(np.asarray(tx.pos, dtype=np.float64)[None, :], n, axis=0)
    d = d0.copy()
    w = np.ones(n)
    s_len = np.zeros(n)
    excl = np.full(n, -1, dtype=np.int32)
    seq = [() for _ in range(n)]
    alive = np.arange(n)
    eta_m = em.eta(geo.materials[:, 0], geo.materials[:, 1], geo.freq)
    pec_m = ~np.isfinite(geo.materials[:, 1])
    R = np.asarray([rx.pos for rx in rxs], dtype=np.float64).reshape(-1, 3)
    dom = 4.0 * np.pi / N
    out = [[] for _ in rxs]
    for k in range(1, params.max_depth + 1):
        if alive.size == 0:
            break
        tri, t = native.closest_hit(o, d, excl, params.tmin, geo.V, geo.F, geo.face, threads=threads)
        hit = tri >= 0
        alive, o, d, U, w, s_len, tri, t = alive[hit], o[hit], d[hit], U[hit], w[hit], s_len[hit], tri[hit], t[hit]
        if alive.size == 0:
            break
        h = o + t[:, None] * d
        s_len = s_len + t
        d_r, n_f, cos_i = em.reflect(d, geo.normal[tri])
        m = geo.tri_mat[tri]
        f = geo.face[tri].astype(np.int32)
        rp, rl = em.fresnel(eta_m[m], cos_i, pec=pec_m[m])
        Sm = S[m]
        for j, r in enumerate(alive):
            seq[r] = seq[r] + (int(f[j]),)
        # (hit, receiver) pairs in front of a scattering face
        v = R[None, :, :] - h[:, None, :]
        front = (np.einsum("mrk,mk->mr", v, n_f) > 0.0) & (Sm > 0.0)[:, None]
        jj, rr = np.nonzero(front)
        if jj.size:
            occ = native.occluded(h[jj], R[rr], f[jj], np.full(jj.size, -1, dtype=np.int32), OCC_EPS,
                                  geo.V, geo.F, geo.face, threads=threads)
            jj, rr = jj[~occ], rr[~occ]
        for j, r in zip(jj.tolist(), rr.tolist()):
            vec = R[r] - h[j]
            r_s = float(np.linalg.norm(vec))
            kv = vec / r_s
            cos_s = float(np.dot(kv, n_f[j]))
            c = Sm[j] * w[j] * np.sqrt(dom * cos_s / np.pi) / r_s
            Es = em.transfer_scattered(U[j], np.repeat(d[j][None], 2, 0), np.repeat(kv[None], 2, 0),
                                       np.repeat(n_f[j][None], 2, 0), np.repeat(rp[j], 2), np.repeat(rl[j], 2))
            thk, phk = em.theta_phi(kv)
            b = np.stack([em.theta_hat(thk, phk), em.phi_hat(phk)])
            L = float(s_len[j] + r_s)
            T = L * c * (b @ Es.T)
            E = ftx[alive[j], 0] * Es[0] + ftx[alive[j], 1] * Es[1]
            frx = em.antenna_field(rxs[r], -kv[None, :])[0]
            a = lam / (4.0 * np.pi) * c * np.dot(frx, E)
            ray = int(idx[alive[j]])
            out[r].append(ScatPath(r, ray, k, seq[alive[j]], complex(a), T, L / C0, L,
                                   _angles(d0[alive[j]]), _angles(-kv), h[j].copy()))
        # specular continuation with the specular share of the power
        U = np.stack([em.transfer(U[:, q], d, d_r, n_f, rp, rl) for q in range(2)], axis=1)
        w = w * np.sqrt(1.0 - Sm * Sm)
        o, d, excl = h, d_r, f
    for lst in out:
        lst.sort(key=lambda p: (p.ray, p.depth))
    return out


def received_power(path_list):
    """Incoherent received power sum |a|^2 over one rx's scattered paths."""
    return float(sum(abs(p.a) ** 2 for p in path_list))
