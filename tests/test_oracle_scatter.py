"""Pins of the diffuse-scattering oracle (oracle.scatter and its use in
oracle.sbr): the SplitMix64 draws equal the published reference outputs; the
cosine-weighted sampler has E[cos] = 2/3, E[cos^2] = 1/2 and no azimuthal
bias; S = 0 leaves the specular map unchanged; and over a perfectly
conducting ground with S = 1 the scattered part of the map (receive patterns V
plus H, i.e. the total power) equals the Lambertian closed form
    g(x) = (lambda/4pi)^2 int_ground (h / s^3) (z_x / (pi r^3)) dA,
s = |p - tx|, r = |x - p| (incident flux through the tilted area element,
re-radiated with radiance proportional to cos(theta_s)), integrated by
quadrature over the region's cells."""
from types import SimpleNamespace

import numpy as np

import scenegen as sg
from oracle import em, sbr, scatter


def test_splitmix64_reference_outputs():
    out = scatter.splitmix64(0, np.arange(3))
    assert [int(x) for x in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    u = scatter.uniform(12345, np.arange(200_000))
    assert 0.0 <= u.min() and u.max() < 1.0 and abs(u.mean() - 0.5) < 3e-3


def test_lambertian_sampler_moments():
    n = np.tile(np.array([[0.3, -0.4, np.sqrt(0.75)]]), (400_000, 1))
    u1 = scatter.uniform(7, np.arange(400_000) * 2)
    u2 = scatter.uniform(7, np.arange(400_000) * 2 + 1)
    d = scatter.lambert_dirs(n, u1, u2)
    c = np.sum(d * n, 1)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-12) and c.min() >= 0.0
    assert abs(c.mean() - 2.0 / 3.0) < 2e-3 and abs((c * c).mean() - 0.5) < 2e-3
    t, b = scatter.tangent_frame(n[:1])
    assert abs(np.mean(d @ t[0])) < 3e-3 and abs(np.mean(d @ b[0])) < 3e-3


def _ground(sigma):
    L = 200.0
    V = np.array([[-L, -L, 0.0], [L, -L, 0.0], [L, L, 0.0], [-L, L, 0.0]], dtype=np.float32)
    F = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    return sg.Scene("ground", V, F, np.zeros(2, dtype=np.int32), np.array([[5.24, sigma]], dtype=np.float32),
                    ["ground"], 3.5e9)


def test_zero_scattering_coefficient_is_specular():
    s = _ground(0.12)
    tx = sg.Device((0.0, 0.0, 10.0))
    grid = sg.Grid(-20.0, -20.0, 2.0, 20, 20, 1.5)
    p = sbr.TraceParams(num_rays=20_000, max_depth=2)
    g0, h0, _ = sbr.coverage(s, tx, p, grid)
    g1, h1, _ = sbr.coverage(s, tx, p, grid, scattering=([0.0], 5))
    assert np.array_equal(h0, h1) and np.array_equal(g0, g1)


def test_lambertian_ground_matches_the_closed_form():
    s = _ground(np.inf)
    h = 10.0
    tx = sg.Device((0.0, 0.0, h))
    grid = sg.Grid(-10.0, -10.0, 2.0, 10, 10, 1.5)
    N = 400_000
    tot = {}
    for D in (0, 1):
        acc = 0.0
        for pol in (sg.POL_V, sg.POL_H):
            rx = SimpleNamespace(yaw=0.0, pitch=0.0, roll=0.0, pattern=em.PATTERN_ISO, pol=pol)
            g, _, _ = sbr.coverage(s, tx, sbr.TraceParams(num_rays=N, max_depth=D), grid, rx_ant=rx,
                                   scattering=([1.0], 99))
            acc += g.sum() * grid.cell ** 2
        tot[D] = acc
    mc = tot[1] - tot[0]
    # quadrature: cell sub-points x, ground points p (fine grid near the axis, coarse outside)
    lam = em.wavelength(s.freq_hz)
    sub = (np.arange(4) + 0.5) / 4 * grid.cell
    xs = (grid.x0 + np.arange(grid.nx)[:, None] * grid.cell + sub[None, :]).ravel()
    ys = (grid.y0 + np.arange(grid.ny)[:, None] * grid.cell + sub[None, :]).ravel()
    X = np.stack(np.meshgrid(xs, ys, indexing="ij"), -1).reshape(-1, 2)
    dA_x = (grid.cell / 4) ** 2
    f = 0.25
    pf = np.arange(-40.0 + f / 2, 40.0, f)
    P_in = np.stack(np.meshgrid(pf, pf, indexing="ij"), -1).reshape(-1, 2)
    c = 2.0
    pc = np.arange(-200.0 + c / 2, 200.0, c)
    P_out = np.stack(np.meshgrid(pc, pc, indexing="ij"), -1).reshape(-1, 2)
    P_out = P_out[(np.abs(P_out) > 40.0).any(1)]
    total = 0.0
    for P, dA in ((P_in, f * f), (P_out, c * c)):
        s3 = (np.sum(P ** 2, 1) + h * h) ** 1.5
        wp = h / s3 * dA
        for k in range(0, X.shape[0], 64):
            x = X[k:k + 64]
            r2 = np.sum((x[:, None, :] - P[None, :, :]) ** 2, -1) + grid.z ** 2
            total += np.sum(wp[None, :] * grid.z / (np.pi * r2 ** 1.5)) * dA_x
    ref = (lam / (4 * np.pi)) ** 2 * total
    print("Monte Carlo %.6e closed form %.6e" % (mc, ref))
    assert abs(mc - ref) < 0.03 * ref
