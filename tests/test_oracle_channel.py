"""Pins of the channel-response oracle (oracle.channel) against closed forms:
a single path has a flat magnitude and a phase that falls by 2 pi spacing tau
per subcarrier (its group delay); two elements half a wavelength apart along
the departure direction differ by pi; a transmitter moving at v along the
departure direction advances the phase by 2 pi v / (lambda fs) per sample;
two paths give the two-ray fading law |H|^2 = |a1|^2 + |a2|^2 +
2 Re(a1 conj(a2) exp(-j 2 pi (f_c + f)(tau1 - tau2)))."""
import numpy as np

from oracle import channel
from oracle.consts import C0

F = 3.5e9
LAM = C0 / F


def test_single_path_flat_magnitude_and_group_delay():
    a, tau = 0.3 - 0.4j, 1.234e-6
    H = channel.cfr([(a, tau, (1.0, 0.5), (2.0, -1.0))], F, 128, 30e3)[0, 0, 0]
    assert np.allclose(np.abs(H), abs(a), rtol=1e-12)
    step = np.angle(H[1:] * np.conj(H[:-1]))
    expected = np.angle(np.exp(-2j * np.pi * 30e3 * tau))
    assert np.allclose(step, expected, atol=1e-9)
    k0 = 64  # f = 0: the carrier phase alone
    assert np.isclose(np.angle(H[k0] / a), np.angle(np.exp(-2j * np.pi * F * tau)), atol=1e-6)


def test_half_wavelength_elements_along_the_departure_direction_differ_by_pi():
    tx_el = [[-LAM / 4, 0.0, 0.0], [LAM / 4, 0.0, 0.0]]
    H = channel.cfr([(1.0, 1e-7, (np.pi / 2, 0.0), (np.pi / 2, np.pi))], F, 4, 30e3, tx_el=tx_el)
    ratio = H[0, 0, 1] / H[0, 0, 0]
    assert np.allclose(ratio, -1.0, atol=1e-12)
    # broadside (departure along +y): no phase difference
    H = channel.cfr([(1.0, 1e-7, (np.pi / 2, np.pi / 2), (np.pi / 2, np.pi))], F, 4, 30e3, tx_el=tx_el)
    assert np.allclose(H[0, 0, 1], H[0, 0, 0], atol=1e-12)


def test_doppler_phase_advance_per_sample():
    v, fs = 30.0, 1e6
    H = channel.cfr([(1.0, 1e-7, (np.pi / 2, 0.0), (np.pi / 2, np.pi))], F, 2, 30e3, v_tx=(v, 0.0, 0.0), T=5, fs=fs)
    step = H[1:, 0, 0, 0] / H[:-1, 0, 0, 0]
    assert np.allclose(step, np.exp(2j * np.pi * v / LAM / fs), atol=1e-12)
    # receiver moving towards the arriving wave adds the same shift
    H2 = channel.cfr([(1.0, 1e-7, (np.pi / 2, 0.0), (np.pi / 2, np.pi))], F, 2, 30e3, v_rx=(-v, 0.0, 0.0), T=5,
                     fs=fs)
    assert np.allclose(H2, H, atol=1e-12)


def test_two_ray_frequency_selective_fading():
    a1, t1, a2, t2 = 1.0 + 0.2j, 1.0e-6, -0.5 + 0.3j, 1.4e-6
    H = channel.cfr([(a1, t1, (1.0, 0.0), (2.0, 0.0)), (a2, t2, (1.2, 0.3), (1.9, 0.1))], F, 128, 30e3)[0, 0, 0]
    f = channel.subcarriers(128, 30e3)
    ref = abs(a1) ** 2 + abs(a2) ** 2 + 2 * np.real(a1 * np.conj(a2) * np.exp(-2j * np.pi * (F + f) * (t1 - t2)))
    assert np.allclose(np.abs(H) ** 2, ref, rtol=1e-9)
    assert channel.nmse(H, H) == 0.0
