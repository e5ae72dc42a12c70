"""Coverage-map region gain and its gradient by central finite differences (FP64).

Test infrastructure: see the package docstring.

A coverage map (Sec. II-A) gives the path gain of one transmitter per cell of a
plane; here G is its sum over a set of cells (a region).  The paper steers a
transmitter's orientation by gradient steps (Sec. III-B) and learns radio
materials by gradient descent (Sec. III-A).  For a fixed lattice of rays the
ray geometry (directions and hit points) depends neither on the materials nor
on the transmitter's orientation: only the field does (the transmit pattern at
launch and the Fresnel coefficients at every reflection), so G is a smooth
function of theta = ((eps_r, sigma) per material, tx yaw, tx pitch).  The
reference gradient is the central difference
    (G(theta + h e_k) - G(theta - h e_k)) / (2 h),  h = rel_h max(|theta_k|, 1),
every evaluation re-tracing the same deterministic lattice.

Parameter order: (eps_r, sigma) per material, then yaw, then pitch.
"""
from __future__ import annotations

import copy
from types import SimpleNamespace

import numpy as np

from . import sbr
from .geom import Geometry


def region_gain(geo, scene, tx, params, grid, region=None, rx_ant=None, threads=None, scattering=None):
    """Sum of the linear path gain over the cells with region != 0 (all cells
    when region is None); ``scattering`` as in oracle.sbr.trace (its draws fix
    every diffuse direction, so G stays smooth in theta)."""
    gain, _, _ = sbr.coverage(scene, tx, params, grid, rx_ant=rx_ant, threads=threads, geo=geo,
                              scattering=scattering)
    if region is None:
        return float(gain.sum())
    return float(gain[np.asarray(region) != 0].sum())


def theta_of(geo, tx):
    return np.concatenate([geo.materials.reshape(-1), [float(tx.yaw), float(tx.pitch)]])


def perturbed(geo, tx, k, delta):
    """(geo', tx') with parameter k of theta shifted by delta."""
    nm = geo.materials.shape[0]
    g2, t2 = geo, tx
    if k < 2 * nm:
        g2 = copy.copy(geo)
        g2.materials = geo.materials.copy()
        g2.materials[k // 2, k % 2] += delta
    else:
        t2 = SimpleNamespace(pos=tuple(float(x) for x in tx.pos), yaw=float(tx.yaw), pitch=float(tx.pitch),
                             roll=float(tx.roll), pattern=tx.pattern, pol=getattr(tx, "pol", 0))
        if k == 2 * nm:
            t2.yaw += delta
        else:
            t2.pitch += delta
    return g2, t2


def region_gain_fd(scene, tx, params, grid, region=None, rx_ant=None, rel_h=1e-4, threads=None, scattering=None):
    """(G, dG/dtheta) with the gradient by central differences."""
    geo = Geometry(scene)
    G0 = region_gain(geo, scene, tx, params, grid, region, rx_ant, threads, scattering)
    theta = theta_of(geo, tx)
    grad = np.empty(theta.size)
    for k in range(theta.size):
        h = rel_h * max(abs(theta[k]), 1.0)
        gp, tp = perturbed(geo, tx, k, +h)
        gm, tm = perturbed(geo, tx, k, -h)
        Gp = region_gain(gp, scene, tp, params, grid, region, rx_ant, threads, scattering)
        Gm = region_gain(gm, scene, tm, params, grid, region, rx_ant, threads, scattering)
        grad[k] = (Gp - Gm) / (2.0 * h)
    return G0, grad
