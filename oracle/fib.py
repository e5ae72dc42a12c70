"""Fibonacci-lattice ray directions (paper Sec. II-B: rays are shot in
directions given by a Fibonacci lattice on the sphere; no formula is given).

Test infrastructure: see the package docstring.

Reading used here (global frame; the transmitter's orientation only affects its
antenna pattern): for ray i of N,
    z_i   = 1 - (2 i + 1) / N
    rho_i = sqrt((1 - z_i)(1 + z_i))
    phi_i = 2 pi frac(i g),  g = (sqrt 5 - 1) / 2,
with frac(i g) evaluated exactly as the 64-bit product i * round(2^64 g)
mod 2^64 divided by 2^64.  Every ray owns the solid angle 4 pi / N (the z_i
split the sphere into equal-area bands).
"""
from __future__ import annotations

import numpy as np

from .consts import GOLDEN_U64


def golden_fraction(idx) -> np.ndarray:
    """frac(i g) as (i * round(2^64 g) mod 2^64) / 2^64, in float64."""
    i = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        h = i * np.uint64(GOLDEN_U64)
    return h.astype(np.float64) * (2.0 ** -64)


def directions(num_rays: int, idx=None) -> np.ndarray:
    """Unit directions (len(idx), 3) of rays idx (default: all) of an N-ray lattice."""
    if idx is None:
        idx = np.arange(num_rays, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    z = 1.0 - (2.0 * idx.astype(np.float64) + 1.0) / float(num_rays)
    rho = np.sqrt((1.0 - z) * (1.0 + z))
    phi = 2.0 * np.pi * golden_fraction(idx)
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def subset(num_rays: int, begin: int = 0, stride: int = 1) -> np.ndarray:
    """Ray indices begin, begin + stride, ... below num_rays."""
    return np.arange(begin, num_rays, stride, dtype=np.int64)
