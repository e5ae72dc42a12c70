"""Parity at the sizes the benchmarks run: the whole urban-canyon map (1e7
rays), a strided sub-lattice of the large-city map on its full 2000 x 2000
grid, the differentiation case at 1e6 rays with all 256 receivers, and map
inference of a surrogate trained on the 200 x 200 surrogate grid, each
against the FP64 oracle."""
import time

import numpy as np
import pytest
import torch

import scenegen as sg
from oracle import geom, grad as ograd, image, mlp as omlp, sbr

from gpu_common import ctx, lib, oracle_params, params, requires_gpu, scene

pytestmark = [pytest.mark.gpu, requires_gpu]


def _say(msg):
    print(msg, flush=True)


def _compare_maps(gain, hits, g_ref, h_ref, n_amb, max_depth, min_cells):
    allowed = 2 * (max_depth + 1) * n_amb
    assert int((hits != h_ref).sum()) <= allowed
    cmp = (h_ref >= 16) & (hits == h_ref)
    assert cmp.sum() >= min_cells
    ddb = np.abs(10 * np.log10(gain[cmp]) - 10 * np.log10(g_ref[cmp]))
    assert ddb.max() < 0.1, ddb.max()
    both = (h_ref > 0) & (hits == h_ref)
    rel = np.abs(gain[both] - g_ref[both]) / g_ref[both]
    assert np.quantile(rel, 0.999) < 1e-4 and int((rel > 1e-3).sum()) <= allowed
    return int(cmp.sum()), float(ddb.max())


def test_urban_full_lattice_map_matches_oracle():
    """The urban-canyon benchmark map: 1e7 rays, 3 reflections, 400 x 400
    cells; the oracle traces the same whole lattice (brute force, FP64)."""
    m = lib()
    w = sg.urban_workload()
    p = params(w)
    out = m.coverage_map(ctx(), scene(w.scene), p, w.tx[0], w.grid)
    gain = out["gain"].cpu().numpy().astype(np.float64)
    hits = out["hits"].cpu().numpy()
    t0 = time.perf_counter()
    g_ref, h_ref, n_amb = sbr.coverage(w.scene, w.tx[0], oracle_params(p), w.grid)
    n, worst = _compare_maps(gain, hits, g_ref, h_ref, n_amb, p.max_depth, 20_000)
    _say("urban 1e7: %d cells with >= 16 hits compared, max %.2e dB, %d ambiguous rays, oracle %.1f s" % (
        n, worst, n_amb, time.perf_counter() - t0))
    assert int(out["ray_bounces"][0]) == p.traced()


def test_city_sublattice_map_matches_oracle_on_full_grid():
    """Large city (about 220k triangles, 28 GHz, TR 38.901 transmitter, five
    reflections) on its full 2000 x 2000 grid of 1 m cells: every 8000th ray
    of the 1e8 lattice.  Hit counts per cell must agree; gains per cell to
    fp32 accumulation error; on 50 m blocks (where cells gather >= 16
    crossings) within 0.1 dB."""
    m = lib()
    w = sg.city_workload()
    p = params(w, ray_begin=17, ray_stride=8000)
    out = m.coverage_map(ctx(), scene(w.scene), p, w.tx[0], w.grid)
    gain = out["gain"].cpu().numpy().astype(np.float64)
    hits = out["hits"].cpu().numpy()
    t0 = time.perf_counter()
    g_ref, h_ref, n_amb = sbr.coverage(w.scene, w.tx[0], oracle_params(p), w.grid)
    _say("city stride 8000: %d crossings, %d ambiguous rays, oracle %.1f s" % (
        int(h_ref.sum()), n_amb, time.perf_counter() - t0))
    allowed = 2 * (p.max_depth + 1) * n_amb
    assert int(h_ref.sum()) > 2000
    assert int((hits != h_ref).sum()) <= allowed
    both = (h_ref > 0) & (hits == h_ref)
    rel = np.abs(gain[both] - g_ref[both]) / g_ref[both]
    assert int((rel > 1e-4).sum()) <= allowed, np.sort(rel)[-5:]
    # 50 m blocks
    B = 50
    G = gain.reshape(2000 // B, B, 2000 // B, B).sum((1, 3))
    GR = g_ref.reshape(2000 // B, B, 2000 // B, B).sum((1, 3))
    H = h_ref.reshape(2000 // B, B, 2000 // B, B).sum((1, 3))
    sel = H >= 16
    assert sel.sum() >= 10
    assert np.max(np.abs(10 * np.log10(G[sel] / GR[sel]))) < 0.1
    assert int(out["ray_bounces"][0]) == p.traced()


def test_differentiation_case_at_full_size():
    """1e6 rays, all 256 receivers, TR 38.901 transmitter at pitch +10 deg:
    every receiver's paths equal the oracle's (its own trace and image
    method), and the power gradient over the 9 parameters equals the oracle's
    central differences to 1e-3 relative."""
    m = lib()
    w = sg.diff_workload()
    assert w.num_rays == 1_000_000 and len(w.rx) == 256
    p = params(w, max_paths_per_rx=64)
    sc = scene(w.scene)
    o = m.compute_paths(ctx(), sc, p, w.tx, w.rx)
    g = geom.Geometry(w.scene)
    t0 = time.perf_counter()
    r = sbr.trace(w.scene, w.tx[0], oracle_params(p), candidates=True, geo=g)
    assert m.last_candidate_count(ctx()) == len(r.candidates)
    op = image.paths(g, w.tx[0], w.rx, r.candidates)
    from test_gpu_paths import _check_paths, _gpu_paths
    gp = _gpu_paths(o)
    n = _check_paths(gp, op)
    _say("differentiation case: %d candidates, %d paths to %d receivers equal the oracle's (%.1f s)" % (
        len(r.candidates), n, sum(1 for x in op if x), time.perf_counter() - t0))
    assert n >= 200
    seqs = [sorted(d, key=lambda k: (len(k), k)) for d in gp]
    fd, used, unstable = ograd.fd_gradient(g, w.tx[0], w.rx, seqs)
    assert used.sum() >= 100
    P0, _ = ograd._powers(g, w.tx[0], w.rx, seqs)
    dLdP = torch.tensor(ograd.dloss_dP(P0, used), dtype=torch.float64, device="cuda")
    gr = m.paths_power_grad(ctx(), sc, p, w.tx[0], w.rx, o["depth"][0], o["faces"][0], dLdP).cpu().numpy()
    scale = np.abs(fd)
    big = scale > 1e-6 * scale.max()
    rel = np.abs(gr - fd)[big] / scale[big]
    _say("gradient: %d receivers used, max rel %.2e" % (int(used.sum()), rel.max()))
    assert rel.max() < 1e-3, (gr, fd)


def test_map_inference_matches_oracle_forward():
    """A surrogate trained on ray-traced maps of the 200 x 200 grid of 2 m
    cells: map inference (f16 MFMA, f16 activations, polynomial GELU in f16)
    against the FP64 oracle forward with the same half-precision weights and
    the polynomial GELU, on every cell of 4 held-out transmitters."""
    m_lib = lib()
    from paper_2303_11103_amd import surrogate as S
    w = sg.urban_workload()
    sc = scene(w.scene)
    grid = sg.Grid(-200.0, -200.0, 2.0, 200, 200, 1.5)
    tx_np = sg.rooftop_tx_positions(w.scene, 260, seed=3)
    maps, mask = S.ray_traced_maps(ctx(), sc, m_lib.TraceParams(w.scene.freq_hz, 3, 2_000_000), tx_np[:256], grid)
    maps = torch.where(mask.bool(), maps, torch.zeros_like(maps))
    tx = torch.tensor(tx_np, device="cuda")
    lo = np.array([-200.0, -200.0, 10.0, -200.0, -200.0])
    hi = np.array([200.0, 200.0, 65.0, 200.0, 200.0])
    mm = S.MLP(ctx(), batch=32768, ff_scale=1.0, ff_scale_cell=4.0, seed=3, center=(lo + hi) / 2,
               half=(hi - lo) / 2, prior=(w.scene.freq_hz, grid.z), ff_rows_tx=8, ff_rows_rel=40, ff_scale_rel=32.0)
    S.train(mm, maps.contiguous(), mask.contiguous(), tx[:256].contiguous(), grid, steps=1500, lr=2e-3, seed=3)
    q = tx[256:260].contiguous()
    pred = mm.predict_maps(q, grid).cpu().numpy().astype(np.float64).reshape(-1)
    theta, Bf = mm.get_params()
    theta = omlp.round_weights_f16(theta.cpu().numpy().astype(np.float64))
    Bf = Bf.cpu().numpy().astype(np.float64)
    ys, xs = np.meshgrid(grid.y0 + (np.arange(grid.ny) + 0.5) * grid.cell,
                         grid.x0 + (np.arange(grid.nx) + 0.5) * grid.cell, indexing="ij")
    qn = q.cpu().numpy().astype(np.float64)
    pts = np.concatenate([np.stack([np.full(xs.size, qn[k, 0]), np.full(xs.size, qn[k, 1]),
                                    np.full(xs.size, qn[k, 2]), xs.reshape(-1), ys.reshape(-1)], 1)
                          for k in range(len(qn))])
    vn = omlp.normalize(pts, (lo + hi) / 2, (hi - lo) / 2)
    ref, _ = omlp.forward(theta, vn, Bf, prior_db=omlp.free_space_db(pts, w.scene.freq_hz, grid.z),
                          act=omlp.gelu_poly)
    d = np.abs(pred - ref)
    span = ref.max() - ref.min()
    _say("map inference vs oracle: %d cells, output span %.1f dB, max |d| %.3f dB, rms %.4f dB, p99.9 %.3f dB" % (
        d.size, span, d.max(), np.sqrt(np.mean(d * d)), np.quantile(d, 0.999)))
    assert span > 30
    assert d.max() < 0.5 and np.sqrt(np.mean(d * d)) < 0.1
