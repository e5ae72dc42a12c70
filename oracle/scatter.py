"""Diffuse scattering for coverage maps (FP64).

Test infrastructure: see the package docstring.

Sec. II-B lists diffuse reflection (scattering) among the interactions of the
ray tracer without giving its model.  The model used here is Lambertian with a
scattering coefficient S per material (energy split: a fraction S^2 of the
reflected power is scattered diffusely, 1 - S^2 stays specular), evaluated by
Monte Carlo inside the shoot-and-bounce estimator: at every hit a uniform u
decides the interaction, diffuse when u < S^2; a diffuse ray leaves in a
cosine-weighted direction around the normal facing the incident side, and
carries the reflected field components (r_perp a_perp, r_par a_par)
re-expressed in its own transverse basis.  The selection probability equals
the power fraction, so both branches carry unscaled fields and the
coverage-map deposit keeps its form; its expectation is the specular map
times (1 - S^2) plus the Lambertian diffuse map.

Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) in its stateless form: draw c of a stream with
seed s is mix(s + (c + 1) g), g = 0x9E3779B97F4A7C15, with
mix(z) = z3 ^ (z3 >> 31), z2 = (z ^ (z >> 30)) 0xBF58476D1CE4E5B9,
z3 = (z2 ^ (z2 >> 27)) 0x94D049BB133111EB (arithmetic mod 2^64); a uniform is
the top 53 bits times 2^-53.  Ray i (lattice index), interaction depth k and
draw j in {0: branch, 1, 2: direction} use c = (i (D + 1) + k) 3 + j with D the
maximum depth.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, c):
    """Draw c (array) of the SplitMix64 stream seeded with seed, uint64."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.asarray(c, dtype=np.uint64) + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        return z ^ (z >> np.uint64(31))


def uniform(seed, c):
    return (splitmix64(seed, c) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def counter(ray_idx, depth, max_depth, draw):
    return (np.asarray(ray_idx, dtype=np.uint64) * np.uint64(max_depth + 1) + np.uint64(depth)) * np.uint64(3) \
        + np.uint64(draw)


def tangent_frame(n):
    """(t, b) completing the unit normals n (m, 3) to right-handed frames:
    t = normalize(n x a), a the coordinate axis least aligned with n (lowest
    index on ties), b = n x t."""
    a = np.zeros_like(n)
    a[np.arange(n.shape[0]), np.argmin(np.abs(n), axis=1)] = 1.0
    t = np.cross(n, a)
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    return t, np.cross(n, t)


def lambert_dirs(n, u1, u2):
    """Cosine-weighted directions around unit normals n (m, 3)."""
    t, b = tangent_frame(n)
    r = np.sqrt(u1)
    ang = 2.0 * np.pi * u2
    z = np.sqrt(1.0 - u1)
    return (r * np.cos(ang))[:, None] * t + (r * np.sin(ang))[:, None] * b + z[:, None] * n
