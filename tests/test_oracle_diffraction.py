"""Pins of the first-order diffraction oracle (oracle/diffraction.py): the
transition function against the Fresnel integrals, the UTD field of a
perfectly conducting half-plane against Sommerfeld's exact solution, the
continuity of the total field across shadow boundaries of a lossy right-angle
wedge, reciprocity, and the wedges of the toy scene."""
import numpy as np
import pytest
from scipy.special import erfc, fresnel
from types import SimpleNamespace

import scenegen as sg
from oracle import diffraction as D, em, geom


def test_transition_function_against_fresnel_integrals_and_limits():
    x = np.concatenate([np.logspace(-8, 4, 200), [0.5, 1.0, 2.0, 6.0]])
    u = np.sqrt(x)
    S, C = fresnel(u * np.sqrt(2.0 / np.pi))   # scipy returns (S, C)
    tail = np.sqrt(np.pi / 8) * (1 - 1j) - np.sqrt(np.pi / 2) * (C - 1j * S)   # int_u^inf exp(-j t^2) dt
    ref = 2j * u * np.exp(1j * x) * tail
    got = D.transition(x)
    big = x > 100
    assert np.max(np.abs(got[~big] - ref[~big])) < 1e-12
    assert np.max(np.abs(got[big] - ref[big])) < 1e-8 * np.max(x)  # ref loses x * eps to exp(jx)
    assert abs(D.transition(1e6) - 1.0) < 1e-5
    # small arguments: F(x) = [sqrt(pi x) - 2 x exp(j pi/4) - (2/3) x^2 exp(-j pi/4)] exp(j (pi/4 + x)) + O(x^2.5)
    for xs in (1e-7, 1e-5):
        small = (np.sqrt(np.pi * xs) - 2 * xs * np.exp(1j * np.pi / 4) - 2 / 3 * xs ** 2 * np.exp(-1j * np.pi / 4)) * \
            np.exp(1j * (np.pi / 4 + xs))
        assert abs(D.transition(xs) - small) < 10 * xs ** 2.5


def _exact_halfplane(k, rho, phi, phip, soft):
    """Sommerfeld's half-plane solution (edge on the z axis, screen at phi = 0),
    incident plane wave exp(j k rho cos(phi - phi')), time factor exp(+j w t)."""
    G = lambda a: 1.0 - 0.5 * erfc(np.exp(1j * np.pi / 4) * a)
    r = np.sqrt(2.0 * k * rho)
    ui = np.exp(1j * k * rho * np.cos(phi - phip)) * G(r * np.cos((phi - phip) / 2))
    ur = np.exp(1j * k * rho * np.cos(phi + phip)) * G(r * np.cos((phi + phip) / 2))
    return ui - ur if soft else ui + ur


def _utd_plane_wave(n, k, rho, phi, phip, R0, Rn, Rgo0, Rgon, pol):
    """GO (incident + face reflections) plus the UTD diffracted field of a
    plane wave at normal incidence on a wedge (2-D, L = rho)."""
    ds, dh = D.coefficients(n, phi, phip, np.pi / 2, rho, k, R0, Rn)
    d = ds if pol == 0 else dh
    u = d * np.exp(-1j * k * rho) / np.sqrt(rho)
    if abs(phi - phip) < np.pi:
        u += np.exp(1j * k * rho * np.cos(phi - phip))
    if phip < np.pi and phi < np.pi - phip:          # reflection off the 0-face (phi = 0)
        u += Rgo0[pol] * np.exp(1j * k * rho * np.cos(phi + phip))
    if phip > (n - 1) * np.pi and phi > 2 * n * np.pi - np.pi - phip:   # off the n-face (phi = n pi)
        u += Rgon[pol] * np.exp(1j * k * rho * np.cos(phi - (2 * n * np.pi - phip)))
    return u


@pytest.mark.parametrize("phip_deg", [60.0, 130.0, 235.0])
def test_pec_half_plane_matches_sommerfeld(phip_deg):
    k = 2 * np.pi
    phip = np.radians(phip_deg)
    pec = ((-1.0, 1.0), (-1.0, 1.0))
    for rho in (8.0, 20.0):
        for pol, soft in ((0, True), (1, False)):
            worst = 0.0
            for phi in np.radians(np.arange(0.5, 360.0, 0.73)):
                if min(abs(phi - phip - np.pi), abs(phi + phip - np.pi), abs(phi + phip - 3 * np.pi)) < 1e-9:
                    continue
                got = _utd_plane_wave(2.0, k, rho, phi, phip, *pec, *pec, pol)
                ref = _exact_halfplane(k, rho, phi, phip, soft)
                worst = max(worst, abs(got - ref))
            # the UTD is the exact solution's expansion to order 1 / (k rho)
            assert worst < 0.6 / (k * rho), (rho, pol, worst)


def test_coefficient_on_a_shadow_boundary_is_the_lit_side_limit():
    """Exactly on a shadow boundary the cotangent is infinite and F vanishes;
    the coefficient takes the limit from the lit side."""
    k, L, n = 2 * np.pi, 10.0, 1.5
    R = ((-0.6 + 0.1j, 0.3 - 0.2j), (-0.5 + 0.05j, 0.4 + 0.1j))
    for phip, phi_b, side in ((np.radians(50.0), np.radians(230.0), -1), (np.radians(50.0), np.radians(130.0), -1),
                              (np.radians(120.0), np.radians(240.0), +1)):
        on = np.array(D.coefficients(n, phi_b, phip, 1.2, L, k, *R))
        near = np.array(D.coefficients(n, phi_b + side * 1e-8, phip, 1.2, L, k, *R))
        assert np.max(np.abs(on - near)) < 1e-6 * np.max(np.abs(on))


@pytest.mark.parametrize("phip_deg", [50.0, 120.0])
def test_lossy_right_angle_wedge_total_field_is_continuous_at_shadow_boundaries(phip_deg):
    """Concrete faces at 3.5 GHz (Luebbers' form): the total field (GO with
    Fresnel reflections plus diffraction) has no jump where the incident or a
    reflected wave is cut off, although each part jumps by O(1) there."""
    n, k, rho = 1.5, 2 * np.pi * 3.5e9 / 299792458.0, 7.0
    eta = em.eta(5.31, 0.09, 3.5e9)
    phip = np.radians(phip_deg)
    R0 = tuple(complex(x) for x in em.fresnel(eta, np.sin(phip)))
    Rgon = tuple(complex(x) for x in em.fresnel(eta, abs(np.sin(n * np.pi - phip))))
    bounds = [phip + np.pi, np.pi - phip, 2 * n * np.pi - np.pi - phip]
    checked = 0
    for b in bounds:
        if not (0.0 < b < n * np.pi):
            continue
        for pol in (0, 1):
            vals = []
            for phi in (b - 1e-10, b + 1e-10):
                Rn = tuple(complex(x) for x in em.fresnel(eta, abs(np.sin(n * np.pi - phi))))
                vals.append(_utd_plane_wave(n, k, rho, phi, phip, R0, Rn, R0, Rgon, pol))
            assert abs(vals[0] - vals[1]) < 1e-6, (b, pol, vals)
            checked += 1
    assert checked == 4


def test_diffraction_is_reciprocal_on_a_perfect_conductor():
    s = sg.make_toy()
    s.materials = np.array([[1.0, np.inf]])
    g = geom.Geometry(s)
    wl = D.wedges(g)
    rng = np.random.default_rng(4)
    done = 0
    for _ in range(400):
        S = rng.uniform([-60, -60, 0.5], [120, 60, 40])
        P = rng.uniform([-60, -60, 0.5], [120, 60, 40])
        for w in wl:
            g1 = D.path_geometry(g, w, S, P)
            g2 = D.path_geometry(g, w, P, S)
            if g1 is None or g2 is None:
                continue
            tx = SimpleNamespace(pos=S, yaw=0.3, pitch=0.1, roll=0.0, pattern=em.PATTERN_DIPOLE, pol=2)
            rx = SimpleNamespace(pos=P, yaw=-0.7, pitch=0.0, roll=0.2, pattern=em.PATTERN_TR38901, pol=1)
            a1, _, L1, _, _ = D.path_coefficients(g, w, tx, rx, *g1)
            a2, _, L2, _, _ = D.path_coefficients(g, w, rx, tx, *g2)
            assert abs(L1 - L2) < 1e-9 * L1
            assert abs(a1 - a2) <= 1e-9 * abs(a1), (a1, a2)
            done += 1
    assert done > 100


def test_toy_scene_wedges_and_a_shadowed_receiver():
    w = sg.toy_workload()
    g = geom.Geometry(w.scene)
    wl = D.wedges(g)
    # 12 box edges minus the 4 on the ground: 4 vertical (15 m) and 4 roof edges (20 and 10 m)
    assert len(wl) == 8
    assert sorted(round(x.length, 9) for x in wl) == [10.0, 10.0, 15.0, 15.0, 15.0, 15.0, 20.0, 20.0]
    assert all(abs(x.n - 1.5) < 1e-12 for x in wl)
    for x in wl:
        assert abs(np.dot(x.t0, x.e)) < 1e-12 and abs(np.dot(x.n0, x.e)) < 1e-12 and abs(np.dot(x.t0, x.n0)) < 1e-12
    # a receiver behind the box, without line of sight: reached round the
    # vertical edge at (30, 5), weaker than free space
    rx = SimpleNamespace(pos=(80.0, 8.0, 1.5), yaw=0.0, pitch=0.0, roll=0.0, pattern=0, pol=0)
    from oracle import native
    assert native.occluded(np.array([w.tx[0].pos], dtype=float), np.array([rx.pos]), np.array([-1]),
                           np.array([-1]), 1e-9, g.V, g.F, g.face)[0]
    p = D.paths(g, w.tx[0], [rx], wl)[0]
    assert len(p) >= 1
    assert any(np.allclose(q.point[:2], (30.0, 5.0)) for q in p)
    d_free = np.linalg.norm(np.asarray(rx.pos) - np.asarray(w.tx[0].pos))
    free = (299792458.0 / w.scene.freq_hz / (4 * np.pi * d_free)) ** 2
    tot = sum(abs(q.a) ** 2 for q in p)
    assert 1e-4 * free < tot < free
    for q in p:
        assert abs(q.tau * 299792458.0 - q.length) < 1e-9 * q.length
        lam = 299792458.0 / w.scene.freq_hz
        ft = em.antenna_field(w.tx[0], np.array([[np.sin(q.aod[0]) * np.cos(q.aod[1]), np.sin(q.aod[0]) * np.sin(
            q.aod[1]), np.cos(q.aod[0])]]))[0]
        # iso V-pol at both ends: a = lambda / (4 pi L) (T[0, 0])
        assert abs(q.a - lam / (4 * np.pi * q.length) * q.T[0, 0]) < 1e-12 * abs(q.a) + 1e-30
        assert np.linalg.norm(ft) > 0.99


@pytest.mark.parametrize("mat", [(5.31, 0.09), (1.0, np.inf)])
def test_total_field_continuous_where_line_of_sight_is_cut_in_3d(mat):
    """A receiver crossing the incident shadow boundary of the box's vertical
    edge at (30, 5): the line-of-sight coefficient jumps to zero, the
    coefficient diffracted by that edge (oblique incidence, full vector
    dyadic with the antenna fields) jumps by the opposite amount."""
    from oracle import image
    s = sg.make_toy()
    s.materials = np.array([mat])
    g = geom.Geometry(s)
    wl = D.wedges(g)
    edge = [w for w in wl if np.allclose(w.a[:2], (30.0, 5.0)) and np.allclose(w.b[:2], (30.0, 5.0))]
    assert len(edge) == 1
    w = edge[0]
    tx = SimpleNamespace(pos=np.array([0.0, 0.0, 10.0]), yaw=0.2, pitch=0.1, roll=0.0, pattern=em.PATTERN_TR38901,
                         pol=2)
    y_b = 5.0 * 80.0 / 30.0            # the tx -> (30, 5) line meets x = 80 there
    tot = []
    for y in (y_b - 1e-7, y_b + 1e-7):
        rx = SimpleNamespace(pos=np.array([80.0, y, 3.0]), yaw=-2.0, pitch=0.0, roll=0.0,
                             pattern=em.PATTERN_DIPOLE, pol=1)
        Q, phip, phi = D.path_geometry(g, w, tx.pos, rx.pos)
        ad = D.path_coefficients(g, w, tx, rx, Q, phip, phi)[0]
        lit = abs(phi - phip) < np.pi
        alos = image.coefficients(g, tx, rx, (), np.stack([tx.pos, rx.pos]))[0] if lit else 0.0
        tot.append((ad, alos))
    (d0, l0), (d1, l1) = tot
    assert abs(l0 - l1) > 0.1 * max(abs(l0), abs(l1))         # line of sight is cut
    assert abs((d0 + l0) - (d1 + l1)) < 1e-4 * abs(l0 - l1)    # the total is not
