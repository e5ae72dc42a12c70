"""Edge cases of the GPU path against the oracle: a one-triangle scene, a
single ray, a map no ray reaches, line-of-sight-only depth, a lattice's last
ray alone, a receiver without paths, the sphere mode without any pair, and
empty or invalid inputs rejected on the host."""
import numpy as np
import pytest
import torch

import scenegen as sg
from oracle import geom, image, sbr

from gpu_common import compare_hits, ctx, lib, oracle_params, params, requires_gpu, scene

pytestmark = [pytest.mark.gpu, requires_gpu]


def _one_triangle():
    m = sg._Mesh()
    m.poly([(-50.0, -50.0, 0.0), (50.0, -50.0, 0.0), (0.0, 60.0, 0.0)], 0)
    V, F, M = m.arrays()
    return sg.Scene("one_triangle", V, F, M, np.array([[5.31, 0.09]], dtype=np.float32), ["concrete"], 3.5e9)


def test_one_triangle_scene_hits_and_paths():
    m = lib()
    s = _one_triangle()
    tx = sg.Device((0.0, 0.0, 12.0))
    p = m.TraceParams(s.freq_hz, 2, 20_000, max_paths_per_rx=4)
    tri, t = m.trace_record(ctx(), scene(s), p, tx)
    orc = sbr.trace(s, tx, oracle_params(p), record=True)
    compared, _ = compare_hits(tri.cpu().numpy(), t.cpu().numpy(), orc)
    assert compared >= 20_000
    rx = [sg.Device((10.0, 5.0, 2.0)), sg.Device((0.0, 0.0, -5.0))]  # the second sits below the plane
    o = m.compute_paths(ctx(), scene(s), p, [tx], rx)
    n = o["num_paths"][0].cpu().numpy()
    g = geom.Geometry(s)
    ref = image.paths(g, tx, rx, [(0,)])
    assert n.tolist() == [len(x) for x in ref] == [2, 0]


def test_single_ray_and_last_ray_of_the_lattice():
    m = lib()
    w = sg.urban_workload()
    for (N, begin, stride) in ((1, 0, 1), (w.num_rays, w.num_rays - 1, 1), (w.num_rays, 17, w.num_rays)):
        p = params(w, num_rays=N, ray_begin=begin, ray_stride=stride)
        assert p.traced() == 1
        tri, t = m.trace_record(ctx(), scene(w.scene), p, w.tx[0])
        orc = sbr.trace(w.scene, w.tx[0], oracle_params(p), record=True)
        compare_hits(tri.cpu().numpy(), t.cpu().numpy(), orc)
        out = m.coverage_map(ctx(), scene(w.scene), p, w.tx[0], w.grid)
        assert int(out["ray_bounces"][0]) == 1


def test_map_that_no_ray_reaches_and_depth_zero():
    m = lib()
    w = sg.toy_workload()
    far = sg.Grid(5000.0, 5000.0, 1.0, 16, 8, 1.5)  # far outside the scene's ground
    out = m.coverage_map(ctx(), scene(w.scene), params(w), w.tx[0], far)
    assert int(out["hits"].sum()) == 0 and float(out["gain"].abs().sum()) == 0.0
    assert torch.all(torch.isneginf(out["gain_db"]))
    p0 = params(w, max_depth=0)
    out = m.coverage_map(ctx(), scene(w.scene), p0, w.tx[0], w.grid)
    g_ref, h_ref, n_amb = sbr.coverage(w.scene, w.tx[0], oracle_params(p0), w.grid)
    assert int((out["hits"].cpu().numpy() != h_ref).sum()) <= 2 * n_amb
    assert out["ray_bounces"].cpu().numpy().tolist() == [p0.traced()]


def test_sphere_mode_without_pairs_keeps_line_of_sight():
    m = lib()
    w = sg.toy_workload()
    # a tiny kappa: no sphere is passed, only the line-of-sight paths remain
    p = params(w, max_paths_per_rx=16, cand_mode=1, sphere_kappa=1e-6)
    o = m.compute_paths(ctx(), scene(w.scene), p, w.tx, w.rx)
    assert m.last_candidate_count(ctx()) == 0
    g = geom.Geometry(w.scene)
    ref = image.paths(g, w.tx[0], w.rx, [])
    assert o["num_paths"][0].cpu().numpy().tolist() == [len(x) for x in ref]


def test_empty_and_invalid_inputs_are_rejected():
    m = lib()
    from paper_2303_11103_amd._lib import RTError
    w = sg.toy_workload()
    with pytest.raises(RTError):
        m.Scene(ctx(), w.scene.V, w.scene.F[:0], w.scene.tri_mat[:0], w.scene.materials)
    with pytest.raises(RTError, match="NULL argument|at least one tx"):  # an empty list arrives as NULL
        m.compute_paths(ctx(), scene(w.scene), params(w), w.tx, [])
    with pytest.raises(RTError, match="cand_mode"):
        m.compute_paths(ctx(), scene(w.scene), params(w, cand_mode=3), w.tx, w.rx)
    with pytest.raises(RTError, match="sphere_kappa"):
        m.compute_paths(ctx(), scene(w.scene), params(w, cand_mode=1, sphere_kappa=0.0), w.tx, w.rx)
    with pytest.raises(RTError, match="ray_begin"):
        m.coverage_map(ctx(), scene(w.scene), params(w, ray_begin=w.num_rays), w.tx[0], w.grid)
