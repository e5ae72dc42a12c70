"""Diffuse (Lambertian) scattering in the shoot-and-bounce kernel against the
FP64 oracle that draws the same SplitMix64 numbers: per-bounce hits of the
scattered rays, the coverage map, the specular limit S = 0, and the argument
checks."""
import numpy as np
import pytest
import torch

import scenegen as sg
from oracle import sbr

from gpu_common import compare_hits, ctx, lib, oracle_params, params, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

S = [0.6, 0.35]   # concrete, glass
SEED = 11


def _scene(m, w, s=S):
    sc = m.Scene.from_scenegen(ctx(), w.scene)  # an instance of its own: scattering is scene state
    sc.set_scattering(s, SEED)
    return sc


def test_scattered_ray_hits_match_oracle():
    m = lib()
    w = sg.urban_workload(num_rays=100_000)
    p = params(w)
    sc = _scene(m, w)
    tri, t = m.trace_record(ctx(), sc, p, w.tx[0])
    orc = sbr.trace(w.scene, w.tx[0], oracle_params(p), record=True, scattering=(S, SEED))
    compared, excluded = compare_hits(tri.cpu().numpy(), t.cpu().numpy(), orc)
    print("compared", compared, "excluded", excluded, flush=True)
    assert compared > 150_000


def test_scattering_coverage_matches_oracle():
    m = lib()
    w = sg.urban_workload(num_rays=400_003)
    p = params(w)
    sc = _scene(m, w)
    out = m.coverage_map(ctx(), sc, p, w.tx[0], w.grid)
    gain = out["gain"].cpu().numpy().astype(np.float64)
    hits = out["hits"].cpu().numpy()
    g_ref, h_ref, n_amb = sbr.coverage(w.scene, w.tx[0], oracle_params(p), w.grid, scattering=(S, SEED))
    allowed = 2 * (p.max_depth + 1) * n_amb
    assert int((hits != h_ref).sum()) <= allowed
    both = (h_ref > 0) & (hits == h_ref)
    rel = np.abs(gain[both] - g_ref[both]) / g_ref[both]
    assert np.quantile(rel, 0.999) < 1e-4 and int((rel > 1e-3).sum()) <= allowed
    # scattering changes the map
    plain = m.coverage_map(ctx(), _scene(m, w, [0.0, 0.0]), p, w.tx[0], w.grid)
    assert int((plain["hits"].cpu().numpy() != hits).sum()) > 1000


def test_zero_coefficients_reproduce_the_specular_map():
    m = lib()
    w = sg.urban_workload(num_rays=200_000)
    p = params(w)
    a = m.coverage_map(ctx(), m.Scene.from_scenegen(ctx(), w.scene), p, w.tx[0], w.grid)
    b = m.coverage_map(ctx(), _scene(m, w, [0.0, 0.0]), p, w.tx[0], w.grid)
    assert torch.equal(a["hits"], b["hits"])
    ga, gb = a["gain"].double(), b["gain"].double()
    assert torch.allclose(ga, gb, rtol=1e-6, atol=0.0)


def test_scattering_argument_errors():
    m = lib()
    w = sg.urban_workload(num_rays=10_000)
    sc = m.Scene.from_scenegen(ctx(), w.scene)
    with pytest.raises(RuntimeError, match="\\[0, 1\\]"):
        sc.set_scattering([0.5, 1.5])
    with pytest.raises(RuntimeError, match="material count"):
        sc.set_scattering([0.5])


def test_coverage_gradient_with_scattering_matches_oracle_central_differences():
    from oracle import covgrad
    m = lib()
    w = sg.diff_workload(num_rays=100_000)
    p = params(w)
    sc = _scene(m, w)
    grid = sg.Grid(-200.0, -200.0, 4.0, 100, 100, 1.5)
    tri, t = m.trace_record(ctx(), sc, p, w.tx[0])
    out = m.coverage_grad(ctx(), sc, p, w.tx[0], grid, tri, t).cpu().numpy()
    G_ref, g_ref = covgrad.region_gain_fd(w.scene, w.tx[0], oracle_params(p), grid, scattering=(S, SEED))
    assert abs(out[0] - G_ref) < 1e-4 * G_ref
    scale = np.abs(g_ref)
    big = scale > 1e-6 * scale.max()
    err = np.abs(out[1:] - g_ref)[big] / scale[big]
    print("gradient gpu", out[1:], "\noracle fd   ", g_ref, "\nrel", err, flush=True)
    assert err.max() < 1e-3


def test_scattered_hits_full_lattice_sampled():
    """The bench configuration (urban, 1e7 rays, 3 bounces) with scattering:
    every traced ray is recorded; a random sample of lattice indices is
    re-traced by the oracle with the same draws."""
    m = lib()
    w = sg.urban_workload()
    p = params(w)
    tri, t = m.trace_record(ctx(), _scene(m, w), p, w.tx[0])
    tri = tri.cpu().numpy()
    t = t.cpu().numpy()
    rng = np.random.default_rng(6)
    pos = np.sort(rng.choice(p.num_rays, size=3000, replace=False))
    total = 0
    for k in range(len(pos) // 1000):
        sub = pos[k * 1000:(k + 1) * 1000]
        orc = sbr.trace(w.scene, w.tx[0], oracle_params(p), record=True, idx=sub, scattering=(S, SEED))
        compared, _ = compare_hits(tri[:, sub], t[:, sub], orc)
        total += compared
    assert total > 4000
