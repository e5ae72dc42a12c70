"""Channel frequency responses of paths (FP64).

Test infrastructure: see the package docstring.

Sec. II-A turns paths into channel impulse responses (CIRs), optionally with
synthetic arrays (one traced antenna per array, the other elements added by
phase shifts under a plane-wave assumption) and with Doppler from device
velocities; Sec. III-A transforms CIRs into frequency responses of an OFDM
system (128 subcarriers, 30 kHz apart).  A path with coefficient a (without
its delay phase), delay tau, departure unit vector k_t (angles of departure)
and arrival unit vector k_r (angles of arrival, pointing from the receiver
towards the arriving wave) contributes, with the e^{+j w t} convention of the
field model, at time t, receive element offset r_j, transmit element offset
r_i and baseband frequency f (offset from the carrier f_c):
    a exp(-j 2 pi (f_c + f) tau) exp(j 2 pi (k_t . r_i + k_r . r_j) / lambda) exp(j 2 pi f_D t),
    f_D = (v_tx . k_t + v_rx . k_r) / lambda,
since an element displaced towards the wave sees it earlier by (k . r)/c and a
device moving along k shortens the path at rate v . k.  Subcarrier k of K has
f = (k - floor(K/2)) spacing.
"""
from __future__ import annotations

import numpy as np

from .consts import C0


def unit(theta, phi):
    return np.array([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])


def subcarriers(K, spacing):
    return (np.arange(K) - K // 2) * float(spacing)


def cfr(paths, freq_hz, K, spacing, tx_el=None, rx_el=None, v_tx=(0.0, 0.0, 0.0), v_rx=(0.0, 0.0, 0.0), T=1,
        fs=1.0):
    """H [T, nr_el, nt_el, K] (complex128) of one (tx, rx) pair.

    ``paths``: iterable of (a complex, tau, (theta_t, phi_t), (theta_r, phi_r)).
    ``tx_el`` / ``rx_el``: element offsets [n][3] in metres (None: one element).
    """
    lam = C0 / freq_hz
    te = np.zeros((1, 3)) if tx_el is None else np.asarray(tx_el, dtype=np.float64).reshape(-1, 3)
    re = np.zeros((1, 3)) if rx_el is None else np.asarray(rx_el, dtype=np.float64).reshape(-1, 3)
    f = subcarriers(K, spacing)
    t = np.arange(T) / float(fs)
    H = np.zeros((T, re.shape[0], te.shape[0], K), dtype=np.complex128)
    for a, tau, aod, aoa in paths:
        kt = unit(*aod)
        kr = unit(*aoa)
        fd = (np.dot(v_tx, kt) + np.dot(v_rx, kr)) / lam
        delay = np.exp(-2j * np.pi * (freq_hz + f) * tau)                     # [K]
        tx_ph = np.exp(2j * np.pi * (te @ kt) / lam)                          # [nt]
        rx_ph = np.exp(2j * np.pi * (re @ kr) / lam)                          # [nr]
        dop = np.exp(2j * np.pi * fd * t)                                     # [T]
        H += a * dop[:, None, None, None] * rx_ph[None, :, None, None] * tx_ph[None, None, :, None] * delay
    return H


def nmse(H, H_ref):
    """Normalised mean squared error sum |H - H_ref|^2 / sum |H_ref|^2."""
    return float(np.sum(np.abs(H - H_ref) ** 2) / np.sum(np.abs(H_ref) ** 2))
