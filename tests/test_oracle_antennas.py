"""Pins of the dipole pattern and the polarisation model of oracle.em.

Short dipole along the local z axis: |F|^2 = 1.5 sin^2(theta), whose mean over
the sphere is 1 (a lossless antenna: directivity 1.5 = 1.76 dBi).
Single-port polarisation C_theta = g cos(zeta), C_phi = g sin(zeta): the V and
H fields are orthogonal to each other and to the direction with equal
magnitude, the +-45 degree ports of a cross-polarised antenna are orthogonal
and each couples to V with cos 45 degrees; an isotropic H-pol antenna, like a
V-pol one, is unchanged by a yaw rotation (phi-hat is invariant under
rotations about z)."""
from types import SimpleNamespace

import numpy as np

from oracle import em


def _dev(pattern=em.PATTERN_ISO, pol=0, yaw=0.0, pitch=0.0, roll=0.0):
    return SimpleNamespace(pattern=pattern, pol=pol, yaw=yaw, pitch=pitch, roll=roll)


def _dirs(n, seed):
    v = np.random.default_rng(seed).normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_dipole_pattern_and_its_unit_mean_power():
    th = np.linspace(0.0, np.pi, 2001)
    d = np.stack([np.sin(th), np.zeros_like(th), np.cos(th)], 1)
    F = em.antenna_field(_dev(em.PATTERN_DIPOLE), d)
    p = np.sum(np.abs(F) ** 2, 1)
    assert np.allclose(p, 1.5 * np.sin(th) ** 2, atol=1e-12)
    # mean over the sphere: (1/2) int p(theta) sin(theta) dtheta (azimuth-symmetric)
    w = np.sin(th)
    mean = 0.5 * np.sum((p * w)[1:] + (p * w)[:-1]) / 2 * (th[1] - th[0])
    assert abs(mean - 1.0) < 1e-6


def test_polarisation_ports_are_orthogonal_with_the_expected_couplings():
    d = _dirs(500, 1)
    for pattern in (em.PATTERN_ISO, em.PATTERN_TR38901, em.PATTERN_DIPOLE):
        kw = dict(pattern=pattern, yaw=0.4, pitch=-0.3, roll=0.2)
        FV, FH = em.antenna_field(_dev(pol=0, **kw), d), em.antenna_field(_dev(pol=1, **kw), d)
        FP, FM = em.antenna_field(_dev(pol=2, **kw), d), em.antenna_field(_dev(pol=3, **kw), d)
        g2 = np.sum(FV * FV, 1)
        assert np.allclose(np.sum(FV * d, 1), 0.0, atol=1e-12)
        assert np.allclose(np.sum(FH * d, 1), 0.0, atol=1e-12)
        assert np.allclose(np.sum(FV * FH, 1), 0.0, atol=1e-12)
        assert np.allclose(np.sum(FH * FH, 1), g2, atol=1e-12)
        assert np.allclose(np.sum(FP * FM, 1), 0.0, atol=1e-12)
        assert np.allclose(np.sum(FP * FV, 1), g2 / np.sqrt(2.0), atol=1e-12)
        assert np.allclose(np.sum(FM * FH, 1), -g2 / np.sqrt(2.0), atol=1e-12)


def test_isotropic_h_pol_field_does_not_depend_on_yaw():
    d = _dirs(200, 2)
    F0 = em.antenna_field(_dev(pol=1), d)
    F1 = em.antenna_field(_dev(pol=1, yaw=1.1), d)
    assert np.allclose(F0, F1, atol=1e-12)
