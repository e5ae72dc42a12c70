"""Received-power loss and its gradient by central finite differences (FP64).

Test infrastructure: see the package docstring.

The paper differentiates channel responses with respect to material
properties (eps_r, sigma) and to transmitter orientation and position
(Sec. I, II) and uses such gradients to learn materials (Sec. III-A) and to
orient a transmitter (Sec. III-B).  Here the differentiated quantity is the
received power of every receiver, P_r = sum_p |a_p|^2 over the paths of rx r
(incoherent sum), and the loss L = (1/R) sum_r 10 log10 P_r over the receivers
in a given set.  The reference gradient is the central difference
(L(theta + h) - L(theta - h)) / (2 h) with h = 1e-4 max(|theta|, 1), computed
with the set of face sequences of every receiver frozen; receivers whose
paths change validity within +-h are reported so that callers can exclude
them.

Parameter order: (eps_r, sigma) per material, tx x, y, z, tx yaw, tx pitch.
"""
from __future__ import annotations

import copy
from types import SimpleNamespace

import numpy as np

from . import image, native
from .consts import C0, OCC_EPS


def _powers(geo, tx, rxs, seqs, check_occlusion=True, scat=None):
    """P_r for frozen face sequences; also a per-rx tuple of validity flags.
    ``scat``: scattering coefficients per material (specular share, see image)."""
    lam = C0 / geo.freq
    P = np.zeros(len(rxs))
    valid = []
    segs, owner = [], []
    geoms = []
    for r, rx in enumerate(rxs):
        vr = []
        for s in seqs[r]:
            X = image.geometry(geo, tx.pos, rx.pos, s)
            vr.append(X is not None)
            if X is not None:
                geoms.append((r, s, X, len(vr) - 1))
        valid.append(vr)
    if check_occlusion and geoms:
        A, B, ea, eb = [], [], [], []
        for gi, (r, s, X, _) in enumerate(geoms):
            fl = (-1,) + tuple(s) + (-1,)
            for k in range(len(s) + 1):
                A.append(X[k])
                B.append(X[k + 1])
                ea.append(fl[k])
                eb.append(fl[k + 1])
                owner.append(gi)
        occ = native.occluded(np.asarray(A), np.asarray(B), np.asarray(ea), np.asarray(eb), OCC_EPS, geo.V, geo.F,
                              geo.face)
        blocked = np.zeros(len(geoms), dtype=bool)
        np.logical_or.at(blocked, np.asarray(owner), occ)
    else:
        blocked = np.zeros(len(geoms), dtype=bool)
    for gi, (r, s, X, j) in enumerate(geoms):
        if blocked[gi]:
            valid[r][j] = False
            continue
        a, _, _, _, _ = image.coefficients(geo, tx, rxs[r], s, X, lam)
        P[r] += abs(a * image.specular_share(geo, s, scat)) ** 2
    return P, [tuple(v) for v in valid]


def loss(P, mask):
    """Mean over the receivers in mask of 10 log10 P_r."""
    return float(np.mean(10.0 * np.log10(P[mask])))


def dloss_dP(P, mask):
    """dL/dP_r of ``loss`` (0 outside mask)."""
    g = np.zeros_like(P)
    g[mask] = 10.0 / np.log(10.0) / (mask.sum() * P[mask])
    return g


def _perturbed(geo, tx, k, delta):
    """(geo', tx') with parameter k shifted by delta."""
    nm = geo.materials.shape[0]
    g2, t2 = geo, tx
    if k < 2 * nm:
        g2 = copy.copy(geo)
        g2.materials = geo.materials.copy()
        g2.materials[k // 2, k % 2] += delta
    else:
        j = k - 2 * nm
        t2 = SimpleNamespace(pos=tuple(float(x) for x in tx.pos), yaw=float(tx.yaw), pitch=float(tx.pitch),
                             roll=float(tx.roll), pattern=tx.pattern, pol=getattr(tx, "pol", 0))
        if j < 3:
            pos = list(t2.pos)
            pos[j] += delta
            t2.pos = tuple(pos)
        elif j == 3:
            t2.yaw += delta
        else:
            t2.pitch += delta
    return g2, t2


def param_values(geo, tx):
    return np.concatenate([geo.materials.reshape(-1), np.asarray(tx.pos, dtype=np.float64),
                           [float(tx.yaw), float(tx.pitch)]])


def fd_gradient(geo, tx, rxs, seqs, mask=None, rel_h=1e-4, scat=None):
    """Central-difference gradient of ``loss`` over the rx in mask.

    ``scat`` (optional): scattering coefficients per material; every
    reflection then keeps its specular share sqrt(1 - S^2).
    Returns (grad, mask_used, unstable) where unstable[r] is True when some
    perturbation changed the validity of one of rx r's paths; such receivers
    are removed from mask_used and the gradient is computed without them.
    """
    P0, v0 = _powers(geo, tx, rxs, seqs, scat=scat)
    if mask is None:
        mask = P0 > 0
    theta = param_values(geo, tx)
    n = theta.size
    unstable = np.zeros(len(rxs), dtype=bool)
    evals = []
    for k in range(n):
        h = rel_h * max(abs(theta[k]), 1.0)
        gp, tp = _perturbed(geo, tx, k, +h)
        gm, tm = _perturbed(geo, tx, k, -h)
        Pp, vp = _powers(gp, tp, rxs, seqs, scat=scat)
        Pm, vm = _powers(gm, tm, rxs, seqs, scat=scat)
        for r in range(len(rxs)):
            if vp[r] != v0[r] or vm[r] != v0[r]:
                unstable[r] = True
        evals.append((h, Pp, Pm))
    used = mask & ~unstable & (P0 > 0)
    grad = np.array([(loss(Pp, used) - loss(Pm, used)) / (2 * h) for (h, Pp, Pm) in evals])
    return grad, used, unstable
