"""First-order edge diffraction (float64): wedges of the mesh, diffraction
points by Keller's law and uniform-theory (UTD) diffraction coefficients.

Test infrastructure: see the package docstring.

Paper Sec. II-B lists first-order diffraction among the interactions and
defers its computation to the documentation it points to, which is not
available here.  The model below is the textbook uniform geometrical theory of
diffraction of Kouyoumjian and Pathak (1974) for a wedge, with Luebbers'
(1984) form for faces of finite conductivity; every reading is recorded here:

* wedge: an edge shared by exactly two triangles of two different faces, not
  lying on the ground (the lowest z of the scene, where the solid continues
  into the ground).  The solid lies in the smaller of the two angles between
  the faces' half-planes (the interior angle alpha, convex objects); wedges
  with alpha >= pi - 1e-6 are dropped.  Exterior angle n pi, n = 2 - alpha / pi.
  The 0-face is the face with the smaller id.
* edge frame: e = unit edge direction (first to second vertex, vertices in
  the order of the first triangle), t0 = unit vector in the 0-face orthogonal
  to e pointing from the edge into the face, n0 = the 0-face normal on the
  exterior side (orthogonal to e and t0, n0 . tn < 0).  The angle of a point X
  about the edge is phi(X) = atan2((X - Q) . n0, (X - Q) . t0) in [0, 2 pi);
  the exterior is 0 <= phi <= n pi.
* diffraction point (Keller): Q on the edge with equal angles between the
  edge and the incident and diffracted rays; with axial coordinates z and
  distances r from the edge line of tx and rx, z_Q = z_tx + (z_rx - z_tx)
  r_tx / (r_tx + r_rx).  A path exists when 0 < z_Q < edge length, tx and rx
  lie strictly inside the exterior (0 < phi', phi < n pi), and both legs are
  unoccluded (open segments, the two wedge faces skipped).
* coefficient, s' = |Q - tx|, s = |rx - Q|, beta0 the angle between edge and
  rays, L = s' s sin^2(beta0) / (s' + s):
      D_{s,h} = -exp(-j pi/4) / (2 n sqrt(2 pi k) sin beta0) *
        [ cot((pi + (phi - phi'))/(2n)) F(k L a+(phi - phi'))
        + cot((pi - (phi - phi'))/(2n)) F(k L a-(phi - phi'))
        + R0 cot((pi - (phi + phi'))/(2n)) F(k L a-(phi + phi'))
        + Rn cot((pi + (phi + phi'))/(2n)) F(k L a+(phi + phi')) ]
  a+-(b) = 2 cos^2((2 pi n N+- - b)/2) with N+- the integer nearest to
  (b +- pi)/(2 pi n); F(x) = 2 j sqrt(x) exp(jx) int_sqrt(x)^inf exp(-j t^2) dt.
  R0, Rn: Fresnel coefficients (r_perp for the soft coefficient D_s, r_par for
  the hard D_h) of the 0-face at the local incidence cosine sin(beta0)
  |sin(phi')|, and of the n-face at sin(beta0) |sin(n pi - phi)|; a perfect
  conductor gives R = -1 (soft) and +1 (hard).
* field: phi_hat(X) = -sin(phi) t0 + cos(phi) n0 at the point's angle,
  beta_hat' = phi_hat(tx) x s_in, beta_hat = phi_hat(rx) x s_out with
  s_in = (Q - tx)/s', s_out = (rx - Q)/s; the diffracted field is
  E(rx) = Dbar . E_in(Q) sqrt(s' / (s (s + s'))) exp(-j k s) with
  Dbar = -beta_hat' beta_hat D_s - phi_hat' phi_hat D_h.
* path: a = lambda / (4 pi) F_rx(-s_out) . Dbar F_tx(s_in) /
  sqrt(s' s (s' + s)) (carrier phase excluded, as for reflected paths),
  tau = (s' + s) / c0, T = [theta_hat, phi_hat](s_out)^T Dbar
  [theta_hat, phi_hat](s_in) (s + s') / sqrt(s' s (s + s')) (so that
  a = lambda / (4 pi (s + s')) F_rx^T T F_tx like every other path), AoD the
  angles of s_in, AoA those of -s_out.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.special import erfc

from . import em, native
from .consts import C0, OCC_EPS


@dataclass
class Wedge:
    a: np.ndarray       # first vertex
    b: np.ndarray       # second vertex
    e: np.ndarray       # unit edge direction
    length: float
    t0: np.ndarray
    n0: np.ndarray
    n: float            # exterior angle / pi
    face0: int
    facen: int


@dataclass
class DiffPath:
    rx: int
    wedge: int
    a: complex
    T: np.ndarray
    tau: float
    length: float
    aod: tuple
    aoa: tuple
    point: np.ndarray


def _into_face(a, e, v):
    """Unit vector orthogonal to e from the edge line through a towards v."""
    w = v - a
    w = w - np.dot(w, e) * e
    return w / np.linalg.norm(w)


def wedges(geo):
    """The scene's wedges (see the module docstring), sorted by (face0, facen,
    first vertex, second vertex)."""
    zmin = float(geo.V[:, 2].min())
    edges = {}
    for k in range(geo.F.shape[0]):
        vid = geo.F[k]
        for i in range(3):
            p = tuple(geo.V[vid[i]])
            q = tuple(geo.V[vid[(i + 1) % 3]])
            key = (p, q) if p < q else (q, p)
            edges.setdefault(key, []).append((k, tuple(geo.V[vid[(i + 2) % 3]]), (p, q)))
    out = []
    for key, tl in edges.items():
        if len(tl) != 2:
            continue
        (k1, v1, pq1), (k2, v2, _) = tl
        f1, f2 = int(geo.face[k1]), int(geo.face[k2])
        if f1 == f2:
            continue
        a, b = np.asarray(pq1[0]), np.asarray(pq1[1])
        if a[2] <= zmin and b[2] <= zmin:
            continue
        length = float(np.linalg.norm(b - a))
        e = (b - a) / length
        u1 = _into_face(a, e, np.asarray(v1))
        u2 = _into_face(a, e, np.asarray(v2))
        alpha = float(np.arccos(np.clip(np.dot(u1, u2), -1.0, 1.0)))
        if alpha >= np.pi - 1e-6:
            continue
        if f1 < f2:
            t0, tn, face0, facen = u1, u2, f1, f2
        else:
            t0, tn, face0, facen = u2, u1, f2, f1
        n0 = np.cross(e, t0)
        if np.dot(n0, tn) > 0:
            n0 = -n0
        out.append(Wedge(a, b, e, length, t0, n0, 2.0 - alpha / np.pi, face0, facen))
    out.sort(key=lambda w: (w.face0, w.facen, tuple(w.a), tuple(w.b)))
    return out


def transition(x):
    """F(x) = 2 j sqrt(x) exp(j x) int_sqrt(x)^inf exp(-j t^2) dt for x >= 0,
    written with the complementary error function of sqrt(x) exp(j pi / 4)."""
    x = np.asarray(x, dtype=np.float64)
    return 1j * np.sqrt(np.pi * x) * np.exp(1j * (x - np.pi / 4)) * erfc(np.exp(1j * np.pi / 4) * np.sqrt(x))


def _a_pm(b, n, sign):
    N = np.rint((b + sign * np.pi) / (2.0 * np.pi * n))
    return 2.0 * np.cos((2.0 * np.pi * n * N - b) / 2.0) ** 2


def _term(kL, n, b, sign):
    """cot((pi + sign b)/(2n)) F(kL a^sign(b)), with its limit on a shadow
    boundary (where the cotangent is infinite and F vanishes)."""
    arg = (np.pi + sign * b) / (2.0 * n)
    a = _a_pm(b, n, sign)
    s = np.sin(arg)
    if abs(s) < 1e-12:
        # (pi + sign b) = 2 pi n N + eps: cot(.) F(.) -> n sqrt(2 pi kL) sgn(eps) exp(j pi/4) as eps -> 0
        N = np.rint((np.pi + sign * b) / (2.0 * np.pi * n))
        eps = (np.pi + sign * b) - 2.0 * np.pi * n * N
        return n * np.sqrt(2.0 * np.pi * kL) * (1.0 if eps >= 0 else -1.0) * np.exp(1j * np.pi / 4)
    return np.cos(arg) / s * transition(kL * a)


def coefficients(n, phi, phip, beta0, L, k, R0, Rn):
    """(D_s, D_h) of the module docstring; R0, Rn = (soft, hard) pairs."""
    kL = k * L
    bm, bp = phi - phip, phi + phip
    t1 = _term(kL, n, bm, +1.0)
    t2 = _term(kL, n, bm, -1.0)
    t3 = _term(kL, n, bp, -1.0)
    t4 = _term(kL, n, bp, +1.0)
    pre = -np.exp(-1j * np.pi / 4) / (2.0 * n * np.sqrt(2.0 * np.pi * k) * np.sin(beta0))
    Ds = pre * (t1 + t2 + R0[0] * t3 + Rn[0] * t4)
    Dh = pre * (t1 + t2 + R0[1] * t3 + Rn[1] * t4)
    return Ds, Dh


def angle_about(w, X, Q):
    u = X - Q
    return float(np.mod(np.arctan2(np.dot(u, w.n0), np.dot(u, w.t0)), 2.0 * np.pi))


def keller_point(w, S, P):
    """Diffraction point on the edge line (axial coordinate, point) or None
    when tx or rx lies on the edge line."""
    zs = float(np.dot(S - w.a, w.e))
    zp = float(np.dot(P - w.a, w.e))
    rs = float(np.linalg.norm(S - w.a - zs * w.e))
    rp = float(np.linalg.norm(P - w.a - zp * w.e))
    if rs < 1e-9 or rp < 1e-9:
        return None
    z = zs + (zp - zs) * rs / (rs + rp)
    return z, w.a + z * w.e


def _reflection(geo, face, cos_i):
    m = geo.face_mat[face]
    eps_r, sigma = geo.materials[m]
    if not np.isfinite(sigma):
        return -1.0 + 0j, 1.0 + 0j
    rp, rl = em.fresnel(em.eta(eps_r, sigma, geo.freq), cos_i)
    return complex(rp), complex(rl)


def path_geometry(geo, w, S, P):
    """(Q, phi', phi) of a geometrically valid diffraction over wedge w
    (before occlusion), or None."""
    kp = keller_point(w, S, P)
    if kp is None:
        return None
    z, Q = kp
    if not (0.0 < z < w.length):
        return None
    phip = angle_about(w, S, Q)
    phi = angle_about(w, P, Q)
    lim = w.n * np.pi
    if not (0.0 < phip < lim and 0.0 < phi < lim):
        return None
    return Q, phip, phi


def path_coefficients(geo, w, tx, rx, Q, phip, phi):
    """(a, T, length, s_in, s_out) of the diffracted path tx -> Q -> rx."""
    S = np.asarray(tx.pos, dtype=np.float64)
    P = np.asarray(rx.pos, dtype=np.float64)
    lam = C0 / geo.freq
    k = 2.0 * np.pi / lam
    sp_vec, s_vec = Q - S, P - Q
    sp, s = float(np.linalg.norm(sp_vec)), float(np.linalg.norm(s_vec))
    s_in, s_out = sp_vec / sp, s_vec / s
    cb = float(np.clip(np.dot(s_in, w.e), -1.0, 1.0))
    beta0 = float(np.arccos(cb))
    sb = np.sin(beta0)
    L = sp * s * sb * sb / (sp + s)
    R0 = _reflection(geo, w.face0, sb * abs(np.sin(phip)))
    Rn = _reflection(geo, w.facen, sb * abs(np.sin(w.n * np.pi - phi)))
    Ds, Dh = coefficients(w.n, phi, phip, beta0, L, k, R0, Rn)
    ph_in = -np.sin(phip) * w.t0 + np.cos(phip) * w.n0
    ph_out = -np.sin(phi) * w.t0 + np.cos(phi) * w.n0
    be_in = np.cross(ph_in, s_in)
    be_out = np.cross(ph_out, s_out)
    Dbar = -Ds * np.outer(be_out, be_in) - Dh * np.outer(ph_out, ph_in)   # E_out = Dbar @ E_in
    amp = 1.0 / np.sqrt(sp * s * (sp + s))
    ftx = em.antenna_field(tx, s_in[None, :])[0]
    frx = em.antenna_field(rx, -s_out[None, :])[0]
    a = lam / (4.0 * np.pi) * np.dot(frx, Dbar @ ftx) * amp
    th0, ph0 = em.theta_phi(s_in)
    th1, ph1 = em.theta_phi(s_out)
    Bin = np.stack([em.theta_hat(th0, ph0), em.phi_hat(ph0)])
    Bout = np.stack([em.theta_hat(th1, ph1), em.phi_hat(ph1)])
    T = Bout @ Dbar @ Bin.T * ((sp + s) * amp)
    return complex(a), T, sp + s, s_in, s_out


def paths(geo, tx, rxs, wl=None, threads=None):
    """First-order diffraction paths for every rx over every wedge; a list
    (per rx) of DiffPath sorted by wedge index (index into ``wedges(geo)``)."""
    wl = wedges(geo) if wl is None else wl
    S = np.asarray(tx.pos, dtype=np.float64)
    cand = []
    for r, rx in enumerate(rxs):
        P = np.asarray(rx.pos, dtype=np.float64)
        for i, w in enumerate(wl):
            g = path_geometry(geo, w, S, P)
            if g is not None:
                cand.append((r, i, g))
    A, B, ea, eb = [], [], [], []
    for r, i, (Q, _, _) in cand:
        P = np.asarray(rxs[r].pos, dtype=np.float64)
        for (x, y) in ((S, Q), (Q, P)):
            A.append(x)
            B.append(y)
            ea.append(wl[i].face0)
            eb.append(wl[i].facen)
    occ = native.occluded(np.asarray(A).reshape(-1, 3), np.asarray(B).reshape(-1, 3), np.asarray(ea),
                          np.asarray(eb), OCC_EPS, geo.V, geo.F, geo.face, threads=threads)
    out = [[] for _ in rxs]
    for c, (r, i, (Q, phip, phi)) in enumerate(cand):
        if occ[2 * c] or occ[2 * c + 1]:
            continue
        a, T, L, s_in, s_out = path_coefficients(geo, wl[i], tx, rxs[r], Q, phip, phi)
        th0, ph0 = em.theta_phi(s_in)
        th1, ph1 = em.theta_phi(-s_out)
        out[r].append(DiffPath(r, i, a, T, L / C0, L, (float(th0), float(ph0)), (float(th1), float(ph1)), Q))
    return out


def coverage(geo, tx, grid, rx_ant=None, wl=None, threads=None):
    """Diffraction part of a coverage map: the path gain of the first-order
    diffracted paths at each cell centre (x0 + (ix + 1/2) cell, y0 + (iy +
    1/2) cell, z), summed incoherently over the wedges, with the receive
    pattern rx_ant (isotropic V-pol when None).  Returns (ny, nx) float64."""
    from types import SimpleNamespace
    wl = wedges(geo) if wl is None else wl
    ant = rx_ant if rx_ant is not None else SimpleNamespace(yaw=0.0, pitch=0.0, roll=0.0, pattern=0, pol=0)
    ys = grid.y0 + (np.arange(grid.ny) + 0.5) * grid.cell
    xs = grid.x0 + (np.arange(grid.nx) + 0.5) * grid.cell
    rxs = [SimpleNamespace(pos=(float(x), float(y), float(grid.z)), yaw=ant.yaw, pitch=ant.pitch, roll=ant.roll,
                           pattern=ant.pattern, pol=getattr(ant, "pol", 0)) for y in ys for x in xs]
    per = paths(geo, tx, rxs, wl, threads=threads)
    return np.array([sum(abs(p.a) ** 2 for p in pl) for pl in per]).reshape(grid.ny, grid.nx)
