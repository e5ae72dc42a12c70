"""Pins of the coverage-map region gain and its finite-difference gradient
(oracle.covgrad) against closed forms.

Ground plane, iso V-pol transmitter and receive pattern, one reflection: the
field of a ray is the transmitter's theta-hat, which lies in the plane of
incidence of a horizontal ground, so after the bounce only the parallel
Fresnel coefficient acts and the receive pattern picks up exactly |r_par|^2
(textbook two-ray model).  Every direct crossing therefore adds its ray-tube
weight w = (lambda/4pi)^2 (4pi/N) / (A |d_z|) and every reflected crossing
w |r_par(eta, cos_i)|^2, with
    d r_par / d eta = cos_i (eta - 2 sin_i^2) / (s (eta cos_i + s)^2),
    s = sqrt(eta - sin_i^2), d eta / d eps_r = 1, d eta / d sigma = -j / (eps0 w),
from differentiating r_par = (eta cos_i - s) / (eta cos_i + s).  Rotating an
untilted V-pol antenna about z leaves theta-hat unchanged: dG/d yaw = 0."""
import numpy as np

import scenegen as sg
from oracle import covgrad, em, sbr
from oracle.consts import EPS0


def _ground():
    L = 200.0
    V = np.array([[-L, -L, 0.0], [L, -L, 0.0], [L, L, 0.0], [-L, L, 0.0]], dtype=np.float32)
    F = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    return sg.Scene("ground", V, F, np.zeros(2, dtype=np.int32), np.array([[5.24, 0.12]], dtype=np.float32),
                    ["concrete"], 3.5e9)


def test_region_gain_and_material_gradient_match_the_two_ray_closed_form():
    scene = _ground()
    tx = sg.Device((0.0, 0.0, 10.0))
    grid = sg.Grid(-40.0, -40.0, 2.0, 40, 40, 1.5)
    params = sbr.TraceParams(num_rays=20_000, max_depth=1)
    region = np.zeros((grid.ny, grid.nx), dtype=np.uint8)
    region[5:30, 10:35] = 1
    G, g = covgrad.region_gain_fd(scene, tx, params, grid, region=region)

    res = sbr.trace(scene, tx, params, grid=grid, record=True)
    lam = em.wavelength(scene.freq_hz)
    scale = (lam / (4 * np.pi)) ** 2 * (4 * np.pi / params.num_rays) / grid.cell ** 2

    def crossings(k):
        o, d, t = res.origins[k], res.dirs[k], res.hit_t[k]
        live = ~np.isnan(o[:, 0])
        ok, ix, iy, _, _, _ = sbr._cross_plane(o[live], d[live], t[live], grid)
        inside = np.zeros(ok.shape, dtype=bool)
        inside[ok] = region[iy[ok].astype(int), ix[ok].astype(int)] != 0
        return np.nonzero(live)[0][inside], d[live][inside]

    rays0, d0 = crossings(0)
    rays1, d1 = crossings(1)
    w0 = scale / np.abs(d0[:, 2])
    w1 = scale / np.abs(d1[:, 2])
    cos_i = -res.dirs[0][rays1, 2]           # ground normal +z faces the downward ray
    sin2 = 1.0 - cos_i ** 2
    eps, sig = float(scene.materials[0, 0]), float(scene.materials[0, 1])
    eta = em.eta(eps, sig, scene.freq_hz)
    s = np.sqrt(eta - sin2)
    r_par = (eta * cos_i - s) / (eta * cos_i + s)
    dr = cos_i * (eta - 2.0 * sin2) / (s * (eta * cos_i + s) ** 2)
    G_ref = w0.sum() + (w1 * np.abs(r_par) ** 2).sum()
    dG_deps = (w1 * 2.0 * np.real(np.conj(r_par) * dr)).sum()
    dG_dsig = (w1 * 2.0 * np.real(np.conj(r_par) * dr * (-1j / (EPS0 * 2 * np.pi * scene.freq_hz)))).sum()
    assert rays1.size > 100
    assert abs(G - G_ref) < 1e-10 * G_ref
    assert abs(g[0] - dG_deps) < 1e-6 * abs(dG_deps), (g[0], dG_deps)
    assert abs(g[1] - dG_dsig) < 1e-6 * abs(dG_dsig), (g[1], dG_dsig)
    assert abs(g[2]) < 1e-9 * G                   # yaw of an untilted V-pol antenna


def test_line_of_sight_only_region_gain_does_not_depend_on_materials():
    scene = _ground()
    tx = sg.Device((0.0, 0.0, 10.0), pitch=0.2, pattern=sg.PATTERN_TR38901)
    grid = sg.Grid(-40.0, -40.0, 4.0, 20, 20, 1.5)
    G, g = covgrad.region_gain_fd(scene, tx, sbr.TraceParams(num_rays=5_000, max_depth=0), grid)
    assert G > 0
    assert np.all(g[:2] == 0.0)
    assert abs(g[3]) > 0.0
