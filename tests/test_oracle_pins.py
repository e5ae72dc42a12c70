"""Pins of the FP64 oracle against closed forms, invariants and brute force.

None of these checks re-types an oracle formula: each compares the oracle with
an independent statement of the same physics or mathematics (textbook closed
forms, identities, exhaustive enumeration, quadrature).
"""
from decimal import Decimal, getcontext
from types import SimpleNamespace

import numpy as np
import pytest

import scenegen as sg
from oracle import em, fib, geom, image, native, sbr
from oracle.consts import C0, EPS0


def _scene(V, F, mats, tri_mat=None, freq=3.5e9):
    V = np.asarray(V, dtype=np.float32)
    F = np.asarray(F, dtype=np.int32)
    tri_mat = np.zeros(len(F), dtype=np.int32) if tri_mat is None else np.asarray(tri_mat, dtype=np.int32)
    return sg.Scene("t", V, F, tri_mat, np.asarray(mats, dtype=np.float32), ["m"] * len(mats), freq)


def _quad(m, pts, mat=0):
    m.poly(pts, mat)


def _ground_scene(half=1000.0, mats=((5.31, 0.09),)):
    m = sg._Mesh()
    m.poly([(-half, -half, 0), (half, -half, 0), (half, half, 0), (-half, half, 0)], 0)
    V, F, M = m.arrays()
    return _scene(V, F, mats, M)


def _dev(pos, **kw):
    return sg.Device(tuple(float(x) for x in pos), **kw)


# ---------------------------------------------------------------- Fibonacci lattice
def test_fibonacci_unit_and_equal_area_bands():
    N = 100_003
    d = fib.directions(N)
    assert np.max(np.abs(np.linalg.norm(d, axis=1) - 1.0)) < 1e-15
    # z_i are the mid-points of N equal-area bands: the count in any cap is exact to +-1
    for z0 in (-0.9, -0.3, 0.0, 0.42, 0.99):
        expected = (1.0 - z0) / 2.0 * N
        assert abs(np.sum(d[:, 2] > z0) - expected) <= 1.0
    # no hemisphere bias in azimuth either (quasi-uniform golden-angle spiral)
    assert np.linalg.norm(d.mean(axis=0)) < 1e-4


def test_fibonacci_golden_fraction_against_decimal():
    getcontext().prec = 60
    g = (Decimal(5).sqrt() - 1) / 2
    for i in (0, 1, 2, 3, 1000, 123_456_789, 99_999_999):
        exact = float((Decimal(i) * g) % 1)
        got = float(fib.golden_fraction([i])[0])
        diff = abs(exact - got)
        assert min(diff, 1.0 - diff) < 1e-11


# ---------------------------------------------------------------- intersection
def _independent_closest(o, d, v0, v1, v2, tmin):
    """Plane crossing + same-side edge tests, written without Moller-Trumbore."""
    n = np.cross(v1 - v0, v2 - v0)
    best_t, best_k = np.inf, -1
    for k in range(v0.shape[0]):
        den = np.dot(d, n[k])
        if abs(den) < 1e-300:
            continue
        t = np.dot(v0[k] - o, n[k]) / den
        if not (t > tmin and t < best_t):
            continue
        p = o + t * d
        c0 = np.dot(np.cross(v1[k] - v0[k], p - v0[k]), n[k])
        c1 = np.dot(np.cross(v2[k] - v1[k], p - v1[k]), n[k])
        c2 = np.dot(np.cross(v0[k] - v2[k], p - v2[k]), n[k])
        if c0 >= 0 and c1 >= 0 and c2 >= 0:
            best_t, best_k = t, k
    return best_k, best_t


def test_closest_hit_matches_independent_test_on_urban():
    s = sg.make_urban(0)
    g = geom.Geometry(s)
    o, d = sg.random_rays(400, seed=7, lo=-250, hi=250, zlo=0.5, zhi=70)
    o, d = o.astype(np.float64), d.astype(np.float64)
    tri, t, margin = native.closest_hit(o, d, np.full(len(o), -1), 1e-4, g.V, g.F, g.face, want_margin=True)
    checked = 0
    for r in range(len(o)):
        if margin[r] < 1e-6:
            continue
        k, tt = _independent_closest(o[r], d[r], g.v0, g.v1, g.v2, 1e-4)
        assert k == tri[r] or (k >= 0 and tri[r] >= 0 and abs(tt - t[r]) < 1e-9 and
                               g.face[k] == g.face[tri[r]] and margin[r] < 1e-3)
        if k >= 0:
            assert abs(tt - t[r]) < 1e-9 * max(1.0, tt)
        checked += 1
    assert checked > 350
    assert np.mean(tri >= 0) > 0.3


def test_closest_hit_excludes_face_and_ties_to_lowest_index():
    # two coincident squares (faces 0 and 1 only differ by material) and one behind
    m = sg._Mesh()
    m.poly([(-1, -1, 0), (1, -1, 0), (1, 1, 0), (-1, 1, 0)], 0)
    m.poly([(-1, -1, 0), (1, -1, 0), (1, 1, 0), (-1, 1, 0)], 1)
    m.poly([(-1, -1, -1), (1, -1, -1), (1, 1, -1), (-1, 1, -1)], 0)
    V, F, M = m.arrays()
    s = _scene(V, F, [(2, 0), (3, 0)], M)
    g = geom.Geometry(s)
    o = np.array([[0.3, 0.2, 5.0]])
    d = np.array([[0.0, 0.0, -1.0]])
    tri, t = native.closest_hit(o, d, [-1], 1e-4, g.V, g.F, g.face)
    assert tri[0] == 0 and abs(t[0] - 5.0) < 1e-12
    tri, t = native.closest_hit(o, d, [g.face[0]], 1e-4, g.V, g.F, g.face)
    assert g.face[tri[0]] == g.face[2] and tri[0] in (2, 3)
    tri, t = native.closest_hit(o, d, [g.face[2]], 1e-4, g.V, g.F, g.face)
    assert tri[0] == 0  # face 2 excluded, coincident squares tie -> lowest index


def test_face_grouping_on_toy_and_urban():
    g = geom.Geometry(sg.make_toy())
    # ground + box floor share the z = 0 plane and the material; roof; 4 walls
    assert g.nfaces == 6
    assert list(g.face) == [0, 0, 0, 0, 1, 1, 2, 2, 3, 3, 4, 4, 5, 5]
    s = sg.make_urban(0)
    gu = geom.Geometry(s)
    # every face is planar: all its vertices lie on its plane
    for f in range(gu.nfaces):
        tris = gu.face_tris[f]
        pts = np.concatenate([gu.v0[tris], gu.v1[tris], gu.v2[tris]])
        assert np.max(np.abs((pts - gu.face_point[f]) @ gu.face_normal[f])) < 1e-9
        assert len(set(gu.tri_mat[tris])) == 1
    # walls of buildings in one row/column share planes; roofs never do
    assert gu.nfaces < 770 // 2


# ---------------------------------------------------------------- Fresnel
def _snell_form(eps, cos_i):
    """Fresnel coefficients written with refractive indices and Snell's law."""
    n2 = np.sqrt(eps + 0j)
    sin_t = np.sqrt(1 - cos_i ** 2) / n2
    cos_t = np.sqrt(1 - sin_t ** 2)
    rs = (cos_i - n2 * cos_t) / (cos_i + n2 * cos_t)
    rp = (n2 * cos_i - cos_t) / (n2 * cos_i + cos_t)
    return rs, rp, n2, cos_t


def test_fresnel_against_snell_form_and_power_balance():
    cos_i = np.linspace(0.02, 1.0, 60)
    for eps in (5.31, 6.27, 2.0, 15.0):
        rp_, rl_ = em.fresnel(eps + 0j, cos_i)
        rs, rp, n2, cos_t = _snell_form(eps, cos_i)
        assert np.max(np.abs(rp_ - rs)) < 1e-13
        assert np.max(np.abs(rl_ - rp)) < 1e-13
        # lossless: reflected + transmitted power = 1 for both polarisations
        ts = 1 + rs
        tp = 2 * cos_i / (n2 * cos_i + cos_t)
        k = (n2 * cos_t / cos_i).real
        assert np.max(np.abs(np.abs(rs) ** 2 + k * np.abs(ts) ** 2 - 1)) < 1e-12
        assert np.max(np.abs(np.abs(rp) ** 2 + k * np.abs(tp) ** 2 - 1)) < 1e-12


def test_fresnel_closed_forms():
    eta = em.eta(5.31, 0.09, 3.5e9)
    assert abs(eta.imag + 0.09 / (EPS0 * 2 * np.pi * 3.5e9)) < 1e-15
    # normal incidence: r_par = -r_perp = (sqrt(eta) - 1)/(sqrt(eta) + 1)
    rp, rl = em.fresnel(eta, 1.0)
    ref = (np.sqrt(eta) - 1) / (np.sqrt(eta) + 1)
    assert abs(rl - ref) < 1e-14 and abs(rp + ref) < 1e-14
    # grazing incidence: both -> -1
    rp, rl = em.fresnel(eta, 1e-9)
    assert abs(rp + 1) < 1e-8 and abs(rl + 1) < 1e-8
    # Brewster angle of a lossless dielectric: tan(theta_B) = sqrt(eps_r) -> r_par = 0
    for eps in (5.31, 6.27):
        tb = np.arctan(np.sqrt(eps))
        rp, rl = em.fresnel(eps + 0j, np.cos(tb))
        assert abs(rl) < 1e-15 and abs(rp) > 0.3
    # lossy: |r_par| has a non-zero minimum near theta_B
    th = np.radians(np.linspace(60, 72, 2401))
    _, rl = em.fresnel(eta, np.cos(th))
    k = np.argmin(np.abs(rl))
    assert abs(np.degrees(th[k]) - np.degrees(np.arctan(np.sqrt(5.31)))) < 0.5
    assert 0.005 < np.abs(rl[k]) < 0.05
    # passivity of lossy materials and perfect conductor
    cs = np.linspace(1e-3, 1, 500)
    for (e, s) in ((5.31, 0.09), (6.27, 0.019), (1.0, 1e7), (3.0, 0.1)):
        rp, rl = em.fresnel(em.eta(e, s, 28e9), cs)
        assert np.all(np.abs(rp) <= 1 + 1e-12) and np.all(np.abs(rl) <= 1 + 1e-12)
    rp, rl = em.fresnel(em.eta(5.0, np.inf, 3.5e9), cs)
    assert np.all(rp == -1) and np.all(rl == 1)


# ---------------------------------------------------------------- antennas
def test_tr38901_pattern_values():
    dev = _dev((0, 0, 0), pattern=em.PATTERN_TR38901)
    def gain_db(th_deg, ph_deg, dv=dev):
        th, ph = np.radians(th_deg), np.radians(ph_deg)
        d = np.array([[np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)]])
        f = em.antenna_field(dv, d)[0]
        return 10 * np.log10(np.sum(np.abs(f) ** 2))
    assert abs(gain_db(90, 0) - 8.0) < 1e-12                 # boresight peak
    assert abs(gain_db(90 + 32.5, 0) - 5.0) < 1e-9            # half the 3 dB beamwidth
    assert abs(gain_db(90, 32.5) - 5.0) < 1e-9
    assert abs(gain_db(90, 65) - (8 - 12)) < 1e-9
    assert abs(gain_db(90, 180) - (8 - 30)) < 1e-9            # front-to-back clip
    assert abs(gain_db(0.0, 0) - (8 - 12 * (90 / 65) ** 2)) < 1e-9
    # positive pitch points the beam below the horizon
    tilted = _dev((0, 0, 0), pattern=em.PATTERN_TR38901, pitch=np.radians(10))
    assert abs(gain_db(100, 0, tilted) - 8.0) < 1e-9
    assert abs(gain_db(80, 0, tilted) - (8.0 - 12 * (20 / 65) ** 2)) < 1e-9
    # yaw turns the beam in azimuth
    turned = _dev((0, 0, 0), pattern=em.PATTERN_TR38901, yaw=np.radians(40))
    assert abs(gain_db(90, 40, turned) - 8.0) < 1e-9


def test_iso_v_field_is_theta_hat_and_yaw_invariant():
    d = fib.directions(1000)
    th, ph = em.theta_phi(d)
    f0 = em.antenna_field(_dev((0, 0, 0)), d)
    assert np.max(np.abs(f0 - em.theta_hat(th, ph))) < 1e-14
    fy = em.antenna_field(_dev((0, 0, 0), yaw=0.7), d)
    assert np.max(np.abs(fy - f0)) < 1e-12


# ---------------------------------------------------------------- paths
def test_free_space_path_is_friis():
    s = _ground_scene(10.0)  # tiny ground far below the link, never in the way
    s.V[:, 2] -= 500.0
    g = geom.Geometry(s)
    tx, rx = _dev((0, 0, 10)), _dev((30, 40, 10))
    P = image.paths(g, tx, [rx], [])[0]
    assert len(P) == 1 and P[0].faces == ()
    lam = C0 / 3.5e9
    assert abs(P[0].a - lam / (4 * np.pi * 50.0)) < 1e-15
    assert abs(P[0].tau - 50.0 / C0) < 1e-20
    assert np.allclose(P[0].T, np.eye(2))
    assert abs(P[0].aod[0] - np.pi / 2) < 1e-12 and abs(P[0].aod[1] - np.arctan2(40, 30)) < 1e-12


@pytest.mark.parametrize("azimuth", [0.0, 0.7, 2.5, -2.0])
def test_two_ray_ground_reflection(azimuth):
    s = _ground_scene()
    g = geom.Geometry(s)
    ht, hr, dist = 25.0, 1.5, 120.0
    tx = _dev((0, 0, ht))
    rx = _dev((dist * np.cos(azimuth), dist * np.sin(azimuth), hr))
    P = image.paths(g, tx, [rx], [(0,)])[0]
    assert [p.faces for p in P] == [(), (0,)]
    d1 = np.hypot(dist, ht - hr)
    d2 = np.hypot(dist, ht + hr)
    lam = C0 / 3.5e9
    eta = em.eta(float(np.float32(5.31)), float(np.float32(0.09)), 3.5e9)  # materials are float32 inputs
    cos_i = (ht + hr) / d2
    rs, rp, _, _ = _snell_form(eta, cos_i)
    assert abs(P[0].length - d1) < 1e-9 and abs(P[1].length - d2) < 1e-9
    assert abs(P[1].T[0, 0] - rp) < 1e-12 and abs(P[1].T[1, 1] - rs) < 1e-12
    assert abs(P[1].T[0, 1]) < 1e-12 and abs(P[1].T[1, 0]) < 1e-12
    assert abs(P[1].a - lam * rp / (4 * np.pi * d2)) < 1e-15
    # reflection point on the ground where the angles of incidence and reflection agree
    X = P[1].points[1]
    assert abs(X[2]) < 1e-12
    assert abs(np.hypot(*X[:2]) - dist * ht / (ht + hr)) < 1e-9


def test_pec_dihedral_corner_reflector():
    m = sg._Mesh()
    m.poly([(0, 0, -50), (0, 100, -50), (0, 100, 50), (0, 0, 50)], 0)    # plane x = 0
    m.poly([(0, 0, -50), (100, 0, -50), (100, 0, 50), (0, 0, 50)], 0)    # plane y = 0
    V, F, M = m.arrays()
    s = _scene(V, F, [(1.0, np.inf)], M)
    g = geom.Geometry(s)
    tx, rx = _dev((10, 20, 5)), _dev((30, 7, 5))
    seqs = image.exhaustive_sequences(g.nfaces, 3)
    P = {p.faces: p for p in image.paths(g, tx, [rx], seqs)[0]}
    lam = C0 / 3.5e9
    # double bounce: image of tx through the corner line x = y = 0 -> (-10, -20, 5)
    L2 = np.linalg.norm(np.array([30, 7, 5]) - np.array([-10, -20, 5]))
    # exactly one order of the two walls reaches rx (the other one misses a wall)
    assert {(), (0,), (1,)} < set(P) and len(set(P) & {(0, 1), (1, 0)}) == 1
    assert not any(len(k) == 3 for k in P)  # a right-angle corner has no triple bounce
    for k in set(P) & {(0, 1), (1, 0)}:
        assert abs(P[k].length - L2) < 1e-9
        # horizontal propagation at vertical PEC walls: V-pol is the perp component, r_perp = -1
        assert abs(P[k].T[0, 0] - 1.0) < 1e-12 and abs(P[k].a - lam / (4 * np.pi * L2)) < 1e-15
    for k in ((0,), (1,)):
        assert abs(P[k].T[0, 0] + 1.0) < 1e-12


def test_pec_parallel_plates_image_series():
    W = 12.0
    m = sg._Mesh()
    m.poly([(-500, 0, -50), (500, 0, -50), (500, 0, 50), (-500, 0, 50)], 0)   # y = 0
    m.poly([(-500, W, -50), (500, W, -50), (500, W, 50), (-500, W, 50)], 0)   # y = W
    V, F, M = m.arrays()
    s = _scene(V, F, [(1.0, np.inf)], M)
    g = geom.Geometry(s)
    yt, yr, dx = 3.0, 8.0, 60.0
    tx, rx = _dev((0, yt, 2)), _dev((dx, yr, 2))
    fa = g.face[0]
    seqs = image.exhaustive_sequences(g.nfaces, 4)
    P = {p.faces: p for p in image.paths(g, tx, [rx], seqs)[0]}
    for K in range(1, 5):
        for start in (0, 1):
            seq = tuple((start + i) % 2 for i in range(K))
            seq = tuple(g.face[2 * f] for f in seq)
            m_ = K // 2
            if (seq[0] == fa):   # first bounce on y = 0
                img = yt + 2 * m_ * W if K % 2 == 0 else -yt - 2 * m_ * W
            else:                # first bounce on y = W
                img = yt - 2 * m_ * W if K % 2 == 0 else 2 * W - yt + 2 * m_ * W
            L = np.hypot(dx, yr - img)
            assert seq in P, seq
            assert abs(P[seq].length - L) < 1e-9
            assert abs(abs(P[seq].a) - C0 / 3.5e9 / (4 * np.pi * L)) < 1e-15


def test_reciprocity_and_specular_geometry_on_urban():
    s = sg.make_urban(0)
    g = geom.Geometry(s)
    w = sg.urban_workload(num_rays=20_000)
    tx = w.tx[0]
    rxs = w.rx[:6]
    r = sbr.trace(s, tx, sbr.TraceParams(20_000, 2), candidates=True, geo=g)
    P = image.paths(g, tx, rxs, r.candidates)
    D = np.diag([1.0, -1.0])
    n_checked = 0
    for ri, plist in enumerate(P):
        back = {q.faces: q for q in image.paths(g, rxs[ri], [tx], [q.faces[::-1] for q in plist])[0]}
        for p in plist:
            X = p.points
            # L = |rx - I_K|
            I = np.asarray(tx.pos, dtype=np.float64)
            for f in p.faces:
                n, q = g.face_normal[f], g.face_point[f]
                I = I - 2 * np.dot(I - q, n) * n
            assert abs(p.length - np.linalg.norm(np.asarray(rxs[ri].pos, dtype=np.float64) - I)) < 1e-8
            # Snell / Fermat: the bisector of the two segment directions at X_k is the normal
            for k, f in enumerate(p.faces, start=1):
                a = (X[k - 1] - X[k]) / np.linalg.norm(X[k - 1] - X[k])
                b = (X[k + 1] - X[k]) / np.linalg.norm(X[k + 1] - X[k])
                assert np.linalg.norm(np.cross(a + b, g.face_normal[f])) < 1e-9
            # reciprocity
            q = back[p.faces[::-1]]
            assert abs(q.a - p.a) < 1e-12 * abs(p.a) + 1e-18
            assert np.max(np.abs(q.T - D @ p.T.T @ D)) < 1e-12
            n_checked += 1
    assert n_checked >= 10 and any(len(p.faces) == 2 for pl in P for p in pl)


def test_heuristic_candidates_subset_of_exhaustive_on_toy():
    w = sg.toy_workload()
    g = geom.Geometry(w.scene)
    r = sbr.trace(w.scene, w.tx[0], sbr.TraceParams(w.num_rays, 1), candidates=True, geo=g)
    Ph = image.paths(g, w.tx[0], w.rx, r.candidates)
    Pe = image.paths(g, w.tx[0], w.rx, image.exhaustive_sequences(g.nfaces, 1))
    for a, b in zip(Ph, Pe):
        sa = {p.faces for p in a}
        sb = {p.faces for p in b}
        assert sa <= sb
    recall = sum(len(a) for a in Ph) / sum(len(b) for b in Pe)
    assert recall == 1.0


# ---------------------------------------------------------------- coverage estimator
def _cell_average(fn, x0, y0, cell, n=64):
    u = (np.arange(n) + 0.5) / n * cell
    X, Y = np.meshgrid(x0 + u, y0 + u)
    return float(np.mean(fn(X, Y)))


def test_coverage_free_space_is_friis_cell_average():
    s = _ground_scene(1.0)
    s.V[:, 2] -= 1000.0
    tx = _dev((0, 0, 10))
    grid = sg.Grid(-40.0, -40.0, 4.0, 20, 20, 1.5)
    N = 2_000_000
    gain, hits, _ = sbr.coverage(s, tx, sbr.TraceParams(N, 0), grid)
    lam = C0 / 3.5e9
    checked = 0
    for iy in range(grid.ny):
        for ix in range(grid.nx):
            if hits[iy, ix] < 200:
                continue
            x0, y0 = grid.x0 + ix * grid.cell, grid.y0 + iy * grid.cell
            ref = (lam / (4 * np.pi)) ** 2 * _cell_average(lambda X, Y: 1 / (X ** 2 + Y ** 2 + 8.5 ** 2), x0, y0, 4.0)
            assert abs(gain[iy, ix] / ref - 1) < 3 / np.sqrt(hits[iy, ix])
            checked += 1
    assert checked > 100


def test_coverage_pec_ground_is_incoherent_two_ray_average():
    s = _ground_scene(2000.0, mats=((1.0, np.inf),))
    tx = _dev((0, 0, 20))
    grid = sg.Grid(-50.0, -50.0, 5.0, 20, 20, 1.5)
    N = 2_000_000
    gain, hits, _ = sbr.coverage(s, tx, sbr.TraceParams(N, 1), grid)
    lam = C0 / 3.5e9
    checked = 0
    for iy in range(grid.ny):
        for ix in range(grid.nx):
            if hits[iy, ix] < 400:
                continue
            x0, y0 = grid.x0 + ix * grid.cell, grid.y0 + iy * grid.cell
            f = lambda X, Y: 1 / (X ** 2 + Y ** 2 + 18.5 ** 2) + 1 / (X ** 2 + Y ** 2 + 21.5 ** 2)
            ref = (lam / (4 * np.pi)) ** 2 * _cell_average(f, x0, y0, 5.0)
            assert abs(gain[iy, ix] / ref - 1) < 3 / np.sqrt(hits[iy, ix] / 2)
            checked += 1
    assert checked > 100


def test_coverage_depth_monotone_and_material_independent_hits():
    w = sg.toy_workload()
    p1 = sbr.TraceParams(w.num_rays, 1)
    p2 = sbr.TraceParams(w.num_rays, 2)
    g1, h1, _ = sbr.coverage(w.scene, w.tx[0], p1, w.grid)
    g2, h2, _ = sbr.coverage(w.scene, w.tx[0], p2, w.grid)
    assert np.all(g2 >= g1) and np.all(h2 >= h1) and h2.sum() > h1.sum()
    s2 = sg.make_toy()
    s2.materials[:] = (2.0, 1.0)
    g3, h3, _ = sbr.coverage(s2, w.tx[0], p1, w.grid)
    assert np.array_equal(h1, h3) and not np.allclose(g1, g3)


def test_coverage_matches_image_method_away_from_edges():
    s = _ground_scene(2000.0)
    g = geom.Geometry(s)
    tx = _dev((0, 0, 20))
    grid = sg.Grid(20.0, 20.0, 1.0, 6, 6, 1.5)
    N = 8_000_000
    gain, hits, _ = sbr.coverage(s, tx, sbr.TraceParams(N, 1, ray_begin=0), grid)
    for (ix, iy) in ((1, 1), (3, 4), (5, 2)):
        c = (grid.x0 + ix + 0.5, grid.y0 + iy + 0.5, 1.5)
        P = image.paths(g, tx, [_dev(c)], [(0,)])[0]
        assert abs(gain[iy, ix] / image.received_power(P) - 1) < 0.05


def test_reception_sphere_scale_on_a_ground_plane():
    """Reception spheres are ray tubes widened by kappa: over a single ground
    plane, kappa = 2 gives every receiver the ground reflection (the lattice's
    rays are no farther apart than the tube width), kappa = 0.05 gives almost
    none; sphere candidates are always a subset of the ray prefixes."""
    s = _ground_scene(300.0)
    g = geom.Geometry(s)
    tx = _dev((0, 0, 30))
    rng = np.random.default_rng(7)
    rx = np.concatenate([rng.uniform(-150, 150, size=(40, 2)), np.full((40, 1), 1.5)], 1)
    p = sbr.TraceParams(50_000, 1)
    wide = sbr.trace(s, tx, p, candidates=True, sphere=(rx, 2.0), geo=g)
    ground = {(int(g.face[0]),)}
    assert all(pairs == ground for pairs in wide.sphere_pairs)
    narrow = sbr.trace(s, tx, p, sphere=(rx, 0.05), geo=g)
    assert sum(len(x) for x in narrow.sphere_pairs) <= 5
    assert all(x <= wide.candidates for x in narrow.sphere_pairs)
