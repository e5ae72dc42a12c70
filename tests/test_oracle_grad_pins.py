"""Pins of the oracle's received-power gradient (central differences) and of
its occlusion test against closed forms.

The gradient pins compare ``oracle.grad.fd_gradient`` with derivatives worked
out by hand from textbook formulas, never with another finite difference:

* free space (Friis, isotropic V-pol at both ends): 10 log10 P = const
  - 20 log10 d, so dL/d tx = -(20 / ln 10) mean_r (tx - rx_r) / d_r^2, and the
  materials and the yaw have no effect;
* a tilted isotropic V-pol transmitter seen along its pitch axis couples with
  cos(pitch), so dL/d pitch = -(20 / ln 10) tan(pitch);
* the TR 38.901 element (Table 7.3-1) seen in its horizontal or vertical
  principal plane: the gain in dB is 8 - 12 (offset / 65 deg)^2, so dL/d yaw
  and dL/d pitch are 24 offset / 65^2 per degree;
* two rays over a ground split into two dielectric halves: P_r = (lambda /
  4 pi)^2 (1 / d1^2 + |r_par|^2 / d2^2) with the derivative of the textbook
  r_par = (eta c - s) / (eta c + s), s = sqrt(eta - sin^2), taken by hand:
  dr_par/d eta = c (eta - 2 sin^2) / (s (eta c + s)^2), d eta/d eps_r = 1 and
  d eta/d sigma = -j / (eps0 omega).  Each half's material acts on one
  receiver only, so a swapped parameter index fails.

The occlusion pins place a wall across a segment (blocked), exclude the wall's
face or stop the segment short of it (free), and check that the image method
drops the line of sight and a ground reflection whose leg crosses the wall,
and keeps both when the wall leaves a gap.
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import em, geom, grad, image, native
from oracle.consts import C0, EPS0, OCC_EPS

LN10 = np.log(10.0)
FREQ = 3.5e9


def _scene(mesh, mats, freq=FREQ):
    V, F, M = mesh.arrays()
    return sg.Scene("t", V, F, M, np.asarray(mats, dtype=np.float32), ["m"] * len(mats), freq)


def _dev(pos, **kw):
    return sg.Device(tuple(float(x) for x in pos), **kw)


def _far_ground():
    """A small ground 500 m below the links: never on any path."""
    m = sg._Mesh()
    m.poly([(-10, -10, -500), (10, -10, -500), (10, 10, -500), (-10, 10, -500)], 0)
    return geom.Geometry(_scene(m, [(5.31, 0.09)]))


def _los(n):
    return [[()] for _ in range(n)]


def test_fd_gradient_free_space_matches_friis_closed_form():
    g = _far_ground()
    tx = _dev((3.0, -4.0, 12.0))
    rxs = [_dev((40.0, 25.0, 1.5)), _dev((-30.0, 60.0, 20.0)), _dev((15.0, -70.0, 5.0))]
    gr, used, unstable = grad.fd_gradient(g, tx, rxs, _los(len(rxs)))
    assert used.all() and not unstable.any()
    t = np.asarray(tx.pos)
    want = np.zeros(3)
    for rx in rxs:
        v = t - np.asarray(rx.pos)
        want += -(20.0 / LN10) * v / np.dot(v, v)
    want /= len(rxs)
    assert np.abs(gr[2:5] - want).max() < 1e-6 * np.abs(want).max()
    assert np.abs(gr[0:2]).max() < 1e-12          # no reflection: materials do not act
    assert abs(gr[5]) < 1e-9                      # iso V-pol: yaw does not act


def test_fd_gradient_pitch_of_tilted_iso_v_is_minus_tan():
    g = _far_ground()
    p0 = 0.3
    tx = _dev((0.0, 0.0, 10.0), pitch=p0)
    rxs = [_dev((0.0, 50.0, 10.0)), _dev((0.0, -35.0, 10.0))]   # along the pitch (y) axis
    gr, used, _ = grad.fd_gradient(g, tx, rxs, _los(len(rxs)))
    assert used.all()
    want = -(20.0 / LN10) * np.tan(p0)
    assert abs(gr[6] - want) < 1e-6 * abs(want)


@pytest.mark.parametrize("offset_deg", [-17.0, 9.0, 31.0])
def test_fd_gradient_tr38901_yaw_in_horizontal_plane(offset_deg):
    g = _far_ground()
    yaw0 = np.radians(5.0)
    az = yaw0 + np.radians(offset_deg)
    tx = _dev((0.0, 0.0, 10.0), yaw=yaw0, pattern=sg.PATTERN_TR38901)
    rx = _dev((60.0 * np.cos(az), 60.0 * np.sin(az), 10.0))
    gr, used, _ = grad.fd_gradient(g, tx, [rx], _los(1))
    assert used.all()
    # G = 8 - 12 ((az - yaw) / 65 deg)^2  =>  dG/d yaw = 24 (az - yaw) / 65^2 per degree
    want = 24.0 * offset_deg / 65.0 ** 2 * (180.0 / np.pi)
    assert abs(gr[5] - want) < 1e-6 * abs(want)


@pytest.mark.parametrize("pitch_deg,depression_deg", [(10.0, 4.0), (10.0, 25.0), (-5.0, 12.0)])
def test_fd_gradient_tr38901_pitch_in_vertical_plane(pitch_deg, depression_deg):
    g = _far_ground()
    p0, e = np.radians(pitch_deg), np.radians(depression_deg)
    tx = _dev((0.0, 0.0, 40.0), pitch=p0, pattern=sg.PATTERN_TR38901)
    r = 80.0
    rx = _dev((r * np.cos(e), 0.0, 40.0 - r * np.sin(e)))
    gr, used, _ = grad.fd_gradient(g, tx, [rx], _los(1))
    assert used.all()
    # positive pitch lowers the boresight: the receiver sits (e - p) below it
    want = 24.0 * (depression_deg - pitch_deg) / 65.0 ** 2 * (180.0 / np.pi)
    assert abs(gr[6] - want) < 1e-6 * abs(want)


def _dr_par_deta(eta, c):
    s = np.sqrt(eta - (1.0 - c * c))
    return c * (eta - 2.0 * (1.0 - c * c)) / (s * (eta * c + s) ** 2)


def _r_par(eta, c):
    s = np.sqrt(eta - (1.0 - c * c))
    return (eta * c - s) / (eta * c + s)


def test_fd_gradient_two_ray_materials_match_fresnel_derivative():
    mats = [(5.31, 0.09), (6.27, 0.019)]
    m = sg._Mesh()
    m.poly([(-1000, -1000, 0), (0, -1000, 0), (0, 1000, 0), (-1000, 1000, 0)], 0)   # x < 0: material 0
    m.poly([(0, -1000, 0), (1000, -1000, 0), (1000, 1000, 0), (0, 1000, 0)], 1)     # x > 0: material 1
    s = _scene(m, mats)
    g = geom.Geometry(s)
    ground = {int(g.tri_mat[k]): int(g.face[k]) for k in range(len(g.F))}
    ht, hr = 25.0, 1.5
    tx = _dev((0.0, 0.0, ht))
    rxs = [_dev((-120.0, 0.0, hr)), _dev((110.0, 40.0, hr))]
    seqs = [[(), (ground[0],)], [(), (ground[1],)]]
    gr, used, unstable = grad.fd_gradient(g, tx, rxs, seqs)
    assert used.all() and not unstable.any()
    lam = C0 / FREQ
    k2 = (lam / (4 * np.pi)) ** 2
    omega = 2 * np.pi * FREQ
    want = np.zeros(4)
    for r, rx in enumerate(rxs):
        dist = np.hypot(*rx.pos[:2])
        d1, d2 = np.hypot(dist, ht - hr), np.hypot(dist, ht + hr)
        er, sig = (float(np.float32(v)) for v in mats[r])      # scene materials are float32
        eta = er - 1j * sig / (EPS0 * omega)
        c = (ht + hr) / d2
        rp = _r_par(eta, c)
        P = k2 * (1.0 / d1 ** 2 + abs(rp) ** 2 / d2 ** 2)
        dP_deta = k2 / d2 ** 2 * 2.0 * np.conj(rp) * _dr_par_deta(eta, c)   # d|r|^2 = 2 Re(conj(r) dr)
        dP_der = float(np.real(dP_deta))
        dP_dsig = float(np.real(dP_deta * (-1j / (EPS0 * omega))))
        w = 10.0 / LN10 / (len(rxs) * P)
        want[2 * r] += w * dP_der
        want[2 * r + 1] += w * dP_dsig
    assert np.all(np.abs(want) > 0)
    assert np.abs(gr[:4] - want).max() < 1e-5 * np.abs(want).max(), (gr[:4], want)
    for k in range(4):
        assert abs(gr[k] - want[k]) < 2e-5 * abs(want[k]), (k, gr[k], want[k])


# ---------------------------------------------------------------- occlusion
def _wall_scene(y0=-5.0, y1=5.0, z0=0.0, z1=20.0, with_ground=True):
    m = sg._Mesh()
    if with_ground:
        m.poly([(-200, -200, 0), (200, -200, 0), (200, 200, 0), (-200, 200, 0)], 0)
    m.poly([(10, y0, z0), (10, y1, z0), (10, y1, z1), (10, y0, z1)], 0)    # wall in the plane x = 10
    return geom.Geometry(_scene(m, [(5.31, 0.09)]))


def _occ(g, A, B, ea=-1, eb=-1):
    return bool(native.occluded(np.asarray([A], float), np.asarray([B], float), np.asarray([ea]), np.asarray([eb]),
                                OCC_EPS, g.V, g.F, g.face)[0])


def test_occluded_reports_a_wall_across_the_segment():
    g = _wall_scene(with_ground=False)
    wall = int(g.face[0])
    assert _occ(g, (0, 0, 10), (20, 0, 10))              # straight through the wall
    assert _occ(g, (20, 3, 2), (0, -4, 17))              # oblique, the other way round
    assert not _occ(g, (0, 0, 10), (20, 0, 10), ea=wall)  # the wall's own face is skipped
    assert not _occ(g, (0, 0, 10), (20, 0, 10), eb=wall)
    assert not _occ(g, (0, 0, 10), (9.5, 0, 10))         # ends before the wall
    assert not _occ(g, (10.5, 0, 10), (20, 0, 10))       # starts behind it
    assert not _occ(g, (0, 8, 10), (20, 8, 10))          # passes beside it
    assert not _occ(g, (0, 0, 25), (20, 0, 25))          # passes above it


def test_image_method_drops_paths_whose_legs_cross_a_wall():
    tx, rx = _dev((0, 0, 10)), _dev((20, 0, 1.5))
    g = _wall_scene()
    ground = int(g.face[0])
    got = [p.faces for p in image.paths(g, tx, [rx], [(ground,)])[0]]
    assert got == []                    # LOS and the ground reflection both cross the wall at x = 10
    g_gap = _wall_scene(y0=3.0, y1=10.0)  # the wall leaves the vertical plane y = 0 free
    got = [p.faces for p in image.paths(g_gap, tx, [rx], [(int(g_gap.face[0]),)])[0]]
    assert got == [(), (int(g_gap.face[0]),)]
    g_high = _wall_scene(z0=12.0, z1=20.0)  # the links pass below the wall
    got = [p.faces for p in image.paths(g_high, tx, [rx], [(int(g_high.face[0]),)])[0]]
    assert got == [(), (int(g_high.face[0]),)]
    g_mid = _wall_scene(z0=6.0, z1=20.0)    # the line of sight crosses x = 10 at z = 5.75: free; the
    got = [p.faces for p in image.paths(g_mid, tx, [rx], [(int(g_mid.face[0]),)])[0]]
    # ground reflection's first leg crosses x = 10 at z = 10 - 10 * 10 / (20 * 10 / 11.5) = 4.25: free too
    assert got == [(), (int(g_mid.face[0]),)]
    g_cut = _wall_scene(z0=5.0, z1=20.0)    # now the line of sight (z = 5.75 at the wall) is blocked
    got = [p.faces for p in image.paths(g_cut, tx, [rx], [(int(g_cut.face[0]),)])[0]]
    assert got == [(int(g_cut.face[0]),)]
