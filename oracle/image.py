"""Image-method paths between a transmitter and receivers (float64).

Test infrastructure: see the package docstring.

Paper Sec. II-B: reflected paths are found with the image method, either by
exhaustive search over sequences of primitives or from candidate sequences
produced by shooting Fibonacci-lattice rays; for each candidate the image
method yields the specular path through the same primitives that ends exactly
at the receiver; duplicates are removed and a line-of-sight path is added.
Sec. II-A: a path is returned as a coefficient a and a delay tau.

Conventions (primitives are faces, see ``geom``):

* images: I_0 = tx, I_k = I_{k-1} - 2 ((I_{k-1} - q_k) . n_k) n_k;
* back-tracing: X_{K+1} = rx and X_k is the crossing of the segment
  X_{k+1} -> I_k with plane k, at parameter t in (0, 1);
* a path is valid when every X_k lies in a triangle of face k (signed edge
  distances >= -1e-9 m), X_{k-1} and X_{k+1} lie strictly on the same side of
  plane k, and no open segment X_k -> X_{k+1} (X_0 = tx) is crossed by a
  triangle outside the faces of its two end points, for segment parameters in
  (1e-9, 1 - 1e-9);
* length L = sum of segment lengths (= |rx - I_K|), tau = L / c0;
* a = lambda / (4 pi L) * F_rx(-d_K) . (R_K ... R_1 F_tx(d_0)), where R_k is
  the reflection operator of ``em.transfer`` at X_k; the carrier phase
  exp(-j 2 pi f tau) is not part of a (it is a function of tau alone);
* T: the 2x2 matrix of R_K ... R_1 from (theta_hat(d_0), phi_hat(d_0)) to
  (theta_hat(d_K), phi_hat(d_K));
* AoD = (theta, phi) of d_0, AoA = (theta, phi) of -d_K, global frame,
  theta = acos(z), phi = atan2(y, x);
* line of sight (K = 0) is included when tx -> rx is unoccluded;
* with scattering coefficients S per material (Sec. II-B diffuse reflections,
  the Lambertian power split of ``oracle.scatter``) a reflection keeps the
  specular share 1 - S^2 of the reflected power: a and T carry the factor
  sqrt(1 - S^2) per reflection (S taken in float32, as stored by the library).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

from . import em, native
from .consts import C0, INFACE_TOL, OCC_EPS


@dataclass
class Path:
    rx: int
    faces: tuple
    a: complex
    T: np.ndarray        # (2, 2) complex
    tau: float
    length: float
    aod: tuple
    aoa: tuple
    points: np.ndarray   # (K + 2, 3): tx, X_1..X_K, rx


def _in_face(geo, f, X):
    """X (3,) lies within tolerance inside some triangle of face f."""
    for k in geo.face_tris[f]:
        v = (geo.v0[k], geo.v1[k], geo.v2[k])
        n = np.cross(v[1] - v[0], v[2] - v[0])
        n = n / np.linalg.norm(n)
        ok = True
        for i in range(3):
            a, b = v[i], v[(i + 1) % 3]
            e = b - a
            dist = np.dot(np.cross(e, X - a), n) / np.linalg.norm(e)
            if dist < -INFACE_TOL:
                ok = False
                break
        if ok:
            return True
    return False


def geometry(geo, tx_pos, rx_pos, faces):
    """Points X_0..X_{K+1} of the specular path through ``faces``, or None
    when the image construction fails (before occlusion)."""
    tx = np.asarray(tx_pos, dtype=np.float64)
    rx = np.asarray(rx_pos, dtype=np.float64)
    K = len(faces)
    imgs = [tx]
    for f in faces:
        n, q = geo.face_normal[f], geo.face_point[f]
        I = imgs[-1]
        imgs.append(I - 2.0 * np.dot(I - q, n) * n)
    X = [None] * (K + 2)
    X[0], X[K + 1] = tx, rx
    for k in range(K, 0, -1):
        f = faces[k - 1]
        n, q = geo.face_normal[f], geo.face_point[f]
        A = X[k + 1]
        den = np.dot(imgs[k] - A, n)
        if den == 0.0:
            return None
        t = np.dot(q - A, n) / den
        if not (0.0 < t < 1.0):
            return None
        X[k] = A + t * (imgs[k] - A)
    for k in range(1, K + 1):
        f = faces[k - 1]
        n, q = geo.face_normal[f], geo.face_point[f]
        sp = np.dot(X[k - 1] - q, n)
        sn = np.dot(X[k + 1] - q, n)
        if not (sp * sn > 0.0):
            return None
        if not _in_face(geo, f, X[k]):
            return None
    return np.asarray(X)


def coefficients(geo, tx, rx, faces, X, lam=None):
    """(a, T, length, d_0, d_K) for a geometrically valid path."""
    lam = lam if lam is not None else C0 / geo.freq
    seg = np.diff(X, axis=0)
    lens = np.linalg.norm(seg, axis=1)
    dirs = seg / lens[:, None]
    L = float(lens.sum())
    eta_m = em.eta(geo.materials[:, 0], geo.materials[:, 1], geo.freq)
    pec_m = ~np.isfinite(geo.materials[:, 1])
    d0 = dirs[0]
    E = em.antenna_field(tx, d0[None, :]).astype(np.complex128)
    th0, ph0 = em.theta_phi(d0)
    B = np.stack([em.theta_hat(th0, ph0), em.phi_hat(ph0)]).astype(np.complex128)  # basis at d_0
    for k, f in enumerate(faces):
        d_in, d_out = dirs[k][None, :], dirs[k + 1][None, :]
        _, n_f, cos_i = em.reflect(d_in, geo.face_normal[f][None, :])
        m = geo.face_mat[f]
        rp, rl = em.fresnel(eta_m[m], cos_i, pec=pec_m[m])
        E = em.transfer(E, d_in, d_out, n_f, rp, rl)
        B = em.transfer(B, np.repeat(d_in, 2, 0), np.repeat(d_out, 2, 0), np.repeat(n_f, 2, 0),
                        np.repeat(rp, 2), np.repeat(rl, 2))
    dK = dirs[-1]
    thK, phK = em.theta_phi(dK)
    out_basis = np.stack([em.theta_hat(thK, phK), em.phi_hat(phK)])
    T = out_basis @ B.T  # T[i, j] = b_i(d_K) . R b_j(d_0)
    frx = em.antenna_field(rx, -dK[None, :])[0]
    a = lam / (4.0 * np.pi * L) * np.dot(frx, E[0])
    return complex(a), T, L, d0, dK


def specular_share(geo, faces, scat):
    """Product of sqrt(1 - S^2) over the reflections of a face sequence."""
    if scat is None:
        return 1.0
    S = np.asarray(scat, dtype=np.float32).astype(np.float64)
    w = 1.0
    for f in faces:
        s = S[geo.face_mat[f]]
        w *= np.sqrt(1.0 - s * s)
    return w


def _angles(d):
    th, ph = em.theta_phi(d)
    return float(th), float(ph)


def paths(geo, tx, rxs, sequences, threads=None, scat=None):
    """Valid paths for every rx and every face sequence (the empty sequence
    is line of sight).  ``sequences`` is an iterable of tuples of face ids;
    ``scat`` (optional) the scattering coefficient per material.  Returns a
    list (per rx) of Path lists sorted by (depth, faces)."""
    seqs = sorted(set(tuple(s) for s in sequences) | {()}, key=lambda s: (len(s), s))
    lam = C0 / geo.freq
    cand = []
    for r, rx in enumerate(rxs):
        for s in seqs:
            X = geometry(geo, tx.pos, rx.pos, s)
            if X is not None:
                cand.append((r, s, X))
    # occlusion of every segment, batched
    A, B, ea, eb, owner = [], [], [], [], []
    for ci, (r, s, X) in enumerate(cand):
        fl = (-1,) + tuple(s) + (-1,)
        for k in range(len(s) + 1):
            A.append(X[k])
            B.append(X[k + 1])
            ea.append(fl[k])
            eb.append(fl[k + 1])
            owner.append(ci)
    occ = native.occluded(np.asarray(A).reshape(-1, 3), np.asarray(B).reshape(-1, 3), np.asarray(ea),
                          np.asarray(eb), OCC_EPS, geo.V, geo.F, geo.face, threads=threads)
    blocked = np.zeros(len(cand), dtype=bool)
    if len(owner):
        np.logical_or.at(blocked, np.asarray(owner), occ)
    out = [[] for _ in rxs]
    for ci, (r, s, X) in enumerate(cand):
        if blocked[ci]:
            continue
        a, T, L, d0, dK = coefficients(geo, tx, rxs[r], s, X, lam)
        if scat is not None:
            ws = specular_share(geo, s, scat)
            a, T = a * ws, T * ws
        out[r].append(Path(r, s, a, T, L / C0, L, _angles(d0), _angles(-dK), X))
    return out


def exhaustive_sequences(nfaces, max_depth):
    """Every face sequence of length 1..max_depth without immediate repeats."""
    out = []
    for K in range(1, max_depth + 1):
        for s in itertools.product(range(nfaces), repeat=K):
            if all(s[i] != s[i + 1] for i in range(K - 1)):
                out.append(s)
    return out


def received_power(path_list):
    """Incoherent received power sum |a|^2 over one rx's paths."""
    return float(sum(abs(p.a) ** 2 for p in path_list))
