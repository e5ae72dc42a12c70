"""Pins of the scattered-path oracle (oracle.scatpaths, Sec. II-B diffuse
reflections) against results it does not compute itself:

* over a perfectly conducting ground with S = 1, the received power of the
  scattered paths summed over V and H receive polarisations (the total power)
  equals the Lambertian closed form
      g(R) = (lambda/4pi)^2 int_ground (h / s^3) (z_R / (pi r^3)) dA,
  s = |p - tx|, r = |R - p|, integrated by quadrature over the ground;
* a receiver placed on the specular continuation of a lattice ray sees a
  scattered path whose field, polarisation and transfer matrix equal those of
  the image-method path through the same faces (oracle.image), times the
  scalar ray-tube factor; through a wall and then the ground the earlier
  reflection carries sqrt(1 - S^2);
* with ground only, the scattered paths are exactly the rays that hit the
  ground (counted from the ray directions in closed form); a wall removes
  exactly the rays whose scattering points it hides (closed-form segment test);
* S = 0 gives no paths, a receiver behind the face gives none, and a
  sub-lattice returns the same paths as the full lattice for its rays.
"""
from types import SimpleNamespace

import numpy as np
import pytest

import scenegen as sg
from oracle import em, fib, image, sbr, scatpaths
from oracle.geom import Geometry


def _scene(quads, mats, freq=3.5e9):
    """Scene of axis-aligned rectangles: quads = [(corners (4, 3), material)]."""
    V, F, M = [], [], []
    for q, m in quads:
        b = len(V)
        V.extend(q)
        F.extend([[b, b + 1, b + 2], [b, b + 2, b + 3]])
        M.extend([m, m])
    return sg.Scene("quads", np.asarray(V, dtype=np.float32), np.asarray(F, dtype=np.int32),
                    np.asarray(M, dtype=np.int32), np.asarray(mats, dtype=np.float32),
                    ["m%d" % i for i in range(len(mats))], freq)


def _ground_quad(L=200.0, m=0):
    return ([[-L, -L, 0.0], [L, -L, 0.0], [L, L, 0.0], [-L, L, 0.0]], m)


def _wall_quad(x, y0, y1, z1, m=1):
    return ([[x, y0, 0.0], [x, y1, 0.0], [x, y1, z1], [x, y0, z1]], m)


def _rx(pos, pol=sg.POL_V, pattern=em.PATTERN_ISO, yaw=0.0, pitch=0.0):
    return SimpleNamespace(pos=tuple(float(v) for v in pos), yaw=yaw, pitch=pitch, roll=0.0, pattern=pattern,
                           pol=pol)


def test_conducting_ground_total_power_matches_the_closed_form():
    s = _scene([_ground_quad()], [[1.0, np.inf]])
    h, R = 10.0, np.array([14.0, 3.0, 6.0])
    tx = sg.Device((0.0, 0.0, h))
    rxs = [_rx(R, sg.POL_V), _rx(R, sg.POL_H)]
    out = scatpaths.paths(s, tx, rxs, sbr.TraceParams(num_rays=60_000, max_depth=1), [1.0])
    tot = scatpaths.received_power(out[0]) + scatpaths.received_power(out[1])
    lam = em.wavelength(s.freq_hz)
    total = 0.0
    # ground quadrature: fine cells within 60 m of the axis, coarse outside
    for lo, hi, c, inner in ((-60.0, 60.0, 0.1, True), (-200.0, 200.0, 1.0, False)):
        g = np.arange(lo + c / 2, hi, c)
        for x in np.array_split(g, 16):
            P = np.stack(np.meshgrid(x, g, indexing="ij"), -1).reshape(-1, 2)
            if not inner:
                P = P[(np.abs(P) > 60.0).any(1)]
            s3 = (np.sum(P ** 2, 1) + h * h) ** 1.5
            r3 = (np.sum((P - R[:2]) ** 2, 1) + R[2] ** 2) ** 1.5
            total += np.sum(h / s3 * R[2] / (np.pi * r3)) * c * c
    ref = (lam / (4 * np.pi)) ** 2 * total
    print("scattered paths %.9e closed form %.9e (%d paths)" % (tot, ref, len(out[0])))
    assert abs(tot - ref) < 1e-4 * ref


def _first_ground_ray(N, h, want):
    """Lattice index of the first downward ray with the given property."""
    d = fib.directions(N)
    for i in range(N):
        if d[i, 2] < -0.2 and want(d[i]):
            return i, d[i]
    raise AssertionError("no such ray")


@pytest.mark.parametrize("pols", [(sg.POL_V, sg.POL_V), (sg.POL_SLANT_P45, sg.POL_SLANT_M45)])
def test_specular_direction_equals_the_image_path(pols):
    S = 0.6
    s = _scene([_ground_quad()], [[5.24, 0.12]])
    geo = Geometry(s)
    txp = np.array([0.0, 0.0, 10.0])
    tx = SimpleNamespace(pos=tuple(txp), yaw=0.3, pitch=0.1, roll=0.0, pattern=em.PATTERN_TR38901, pol=pols[0])
    N = 2000
    i, d = _first_ground_ray(N, 10.0, lambda v: v[0] > 0.3)
    hpt = txp + (-txp[2] / d[2]) * d
    dr = d * np.array([1.0, 1.0, -1.0])
    rx = _rx(hpt + 25.0 * dr, pols[1], em.PATTERN_DIPOLE, yaw=2.0, pitch=-0.2)
    sc = scatpaths.paths(s, tx, [rx], sbr.TraceParams(num_rays=N, max_depth=1), [S])[0]
    p = [q for q in sc if q.ray == i]
    assert len(p) == 1 and p[0].depth == 1
    p = p[0]
    im = image.paths(geo, tx, [rx], [(0,)])[0]
    im = [q for q in im if q.faces == (0,)]
    assert len(im) == 1
    im = im[0]
    assert np.allclose(p.point, im.points[1], atol=1e-9)
    r_s = np.linalg.norm(np.asarray(rx.pos) - p.point)
    cos_s = -d[2]
    c = float(np.float32(S)) * np.sqrt(4 * np.pi / N * cos_s / np.pi) / r_s   # S is stored in float32
    assert abs(p.length - im.length) < 1e-9 and abs(p.tau - im.tau) < 1e-15
    assert abs(p.a - p.length * c * im.a) < 1e-9 * abs(p.a)
    assert np.allclose(p.T, c * p.length * im.T, rtol=0, atol=1e-9 * np.abs(p.T).max())
    assert np.allclose(p.aod, im.aod, atol=1e-9) and np.allclose(p.aoa, im.aoa, atol=1e-9)


def test_second_hit_carries_the_specular_share_of_the_first():
    Sw, Sg = 0.4, 0.7
    s = _scene([_ground_quad(), _wall_quad(20.0, -200.0, 200.0, 60.0)], [[5.24, 0.12], [3.0, 0.02]])
    geo = Geometry(s)
    txp = np.array([0.0, 0.0, 10.0])
    tx = SimpleNamespace(pos=tuple(txp), yaw=0.0, pitch=0.0, roll=0.0, pattern=em.PATTERN_ISO, pol=sg.POL_SLANT_P45)
    N = 4000
    # a ray that meets the wall below 10 m and comes down to the ground at x in (0, 20)
    def ok(v):
        t = 20.0 / v[0] if v[0] > 0 else -1.0
        return t > 0 and 0.0 < txp[2] + t * v[2] and txp[2] + t * v[2] < 8.0 and abs(t * v[1]) < 30.0
    i, d = _first_ground_ray(N, 10.0, ok)
    t1 = 20.0 / d[0]
    h1 = txp + t1 * d
    d1 = d * np.array([-1.0, 1.0, 1.0])
    t2 = -h1[2] / d1[2]
    h2 = h1 + t2 * d1
    assert 0.0 < h2[0] < 20.0
    d2 = d1 * np.array([1.0, 1.0, -1.0])
    rx = _rx(h2 + 4.0 * d2, sg.POL_SLANT_M45)
    mats = [Sg, Sw]
    sc = scatpaths.paths(s, tx, [rx], sbr.TraceParams(num_rays=N, max_depth=2), mats)[0]
    p = [q for q in sc if q.ray == i and q.depth == 2]
    assert len(p) == 1
    p = p[0]
    wall_face, ground_face = geo.face[2], geo.face[0]
    assert p.faces == (wall_face, ground_face)
    im = [q for q in image.paths(geo, tx, [rx], [(wall_face, ground_face)])[0] if q.faces == (wall_face, ground_face)]
    assert len(im) == 1
    im = im[0]
    r_s = np.linalg.norm(np.asarray(rx.pos) - p.point)
    c = float(np.float32(Sg)) * np.sqrt(1.0 - float(np.float32(Sw)) ** 2) * np.sqrt(4 * np.pi / N * (-d1[2]) / np.pi) / r_s
    assert abs(p.a - p.length * c * im.a) < 1e-9 * abs(p.a)
    assert np.allclose(p.T, c * p.length * im.T, rtol=0, atol=1e-9 * np.abs(p.T).max())
    # the specular path itself keeps sqrt(1 - S^2) per reflection
    ims = [q for q in image.paths(geo, tx, [rx], [(wall_face, ground_face)], scat=mats)[0]
           if q.faces == (wall_face, ground_face)][0]
    share = np.sqrt(1.0 - float(np.float32(Sw)) ** 2) * np.sqrt(1.0 - float(np.float32(Sg)) ** 2)
    assert abs(ims.a - share * im.a) < 1e-12 * abs(im.a)


def test_ground_paths_are_the_rays_that_hit_the_ground_and_a_wall_hides_its_shadow():
    L = 200.0
    txp = np.array([0.0, 0.0, 10.0])
    tx = sg.Device(tuple(txp))
    R = np.array([-30.0, 10.0, 2.0])
    N = 3000
    d = fib.directions(N)
    t = np.where(d[:, 2] < 0, -txp[2] / np.where(d[:, 2] < 0, d[:, 2], -1.0), 1e9)
    hp = txp + t[:, None] * d
    down = (d[:, 2] < 0) & (np.abs(hp[:, 0]) < L) & (np.abs(hp[:, 1]) < L)
    s = _scene([_ground_quad(L)], [[5.24, 0.12]])
    out = scatpaths.paths(s, tx, [_rx(R)], sbr.TraceParams(num_rays=N, max_depth=1), [0.5])[0]
    assert [p.ray for p in out] == list(np.nonzero(down)[0])
    # a wall x = -20 (|y| < 15, z < 12) between the receiver and part of the ground;
    # it also stops the rays that meet it first
    s2 = _scene([_ground_quad(L), _wall_quad(-20.0, -15.0, 15.0, 12.0)], [[5.24, 0.12], [3.0, 0.02]])
    out2 = scatpaths.paths(s2, tx, [_rx(R)], sbr.TraceParams(num_rays=N, max_depth=1), [0.5, 0.0])[0]

    def crosses_wall(a, b):
        if (a[0] + 20.0) * (b[0] + 20.0) >= 0.0:
            return False
        u = (-20.0 - a[0]) / (b[0] - a[0])
        y, z = a[1] + u * (b[1] - a[1]), a[2] + u * (b[2] - a[2])
        return abs(y) < 15.0 and 0.0 < z < 12.0

    want = [i for i in np.nonzero(down)[0] if not crosses_wall(txp, hp[i]) and not crosses_wall(hp[i], R)]
    got = [p.ray for p in out2]
    assert got == want and len(want) < int(down.sum())


def test_zero_coefficient_receiver_behind_and_sublattice():
    s = _scene([_ground_quad()], [[5.24, 0.12]])
    tx = sg.Device((0.0, 0.0, 10.0))
    p = sbr.TraceParams(num_rays=2000, max_depth=2)
    assert scatpaths.paths(s, tx, [_rx((5.0, 5.0, 2.0))], p, [0.0])[0] == []
    assert scatpaths.paths(s, tx, [_rx((5.0, 5.0, -2.0))], p, [0.8])[0] == []
    full = scatpaths.paths(s, tx, [_rx((5.0, 5.0, 2.0))], p, [0.8])[0]
    sub = scatpaths.paths(s, tx, [_rx((5.0, 5.0, 2.0))],
                          sbr.TraceParams(num_rays=2000, max_depth=2, ray_begin=1, ray_stride=3), [0.8])[0]
    by_ray = {(q.ray, q.depth): q for q in full}
    assert len(sub) > 0 and all(q.ray % 3 == 1 for q in sub)
    assert len(sub) == sum(1 for q in full if q.ray % 3 == 1)
    for q in sub:
        ref = by_ray[(q.ray, q.depth)]
        assert q.a == ref.a and q.tau == ref.tau
