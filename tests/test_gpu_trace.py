"""GPU parity of ray generation, closest-hit tracing and coverage maps
against the FP64 oracle (all calls go through the C ABI)."""
import numpy as np
import pytest
import torch

import scenegen as sg
from oracle import fib, geom, sbr

from gpu_common import compare_hits, ctx, lib, oracle_params, params, requires_gpu, scene

pytestmark = [pytest.mark.gpu, requires_gpu]


def test_fibonacci_directions_match_oracle():
    m = lib()
    for (N, b, s) in ((1, 0, 1), (1000, 0, 1), (10_000_000, 3, 997), (100_000_000, 99_999_000, 1)):
        d = m.fibonacci_directions(ctx(), N, b, s).cpu().numpy()
        ref = fib.directions(N, fib.subset(N, b, s))
        assert d.shape == ref.shape
        assert np.max(np.abs(d - ref)) < 4e-15


def test_scene_faces_match_oracle_grouping():
    for s in (sg.make_toy(), sg.make_urban(0), sg.make_city(0, blocks=8)):
        sc = scene(s)
        ref, nf = geom.face_ids(s.V, s.F, s.tri_mat)
        assert np.array_equal(sc.face_ids(), ref)
        info = sc.info()
        assert info["num_faces"] == nf and info["num_triangles"] == s.nt
        assert info["bvh_depth"] <= 30


@pytest.mark.parametrize("case", ["toy", "urban_stride", "urban_full_small", "city_stride", "city_full_stride",
                                  "city_over_2_18_triangles"])
def test_hits_match_oracle(case):
    m = lib()
    if case == "toy":
        w = sg.toy_workload()
        p = params(w)
    elif case == "urban_stride":
        w = sg.urban_workload()
        p = params(w, ray_begin=7, ray_stride=61)       # 163 935 rays of the 1e7 lattice
    elif case == "urban_full_small":
        w = sg.urban_workload(num_rays=150_001)          # whole lattice: coherent band order on
        p = params(w)
    elif case == "city_stride":
        w = sg.city_workload(num_rays=100_000_000, blocks=12)
        p = params(w, ray_begin=11, ray_stride=2003)     # 49 925 rays of the 1e8 lattice, 5 bounces
    elif case == "city_full_stride":
        w = sg.city_workload()                           # the full large city: 50x50 blocks, ~220k triangles
        p = params(w, ray_begin=13, ray_stride=40009)    # 2 500 rays of the 1e8 lattice, 5 bounces
    else:
        # more than 2^18 triangles: leaf codes use every bit, so the traversal
        # keeps no entry distances in the references to leaves
        w = sg.city_workload(blocks=56)
        assert w.scene.nt > (1 << 18)
        p = params(w, ray_begin=17, ray_stride=40009)
    tri, t = m.trace_record(ctx(), scene(w.scene), p, w.tx[0])
    orc = sbr.trace(w.scene, w.tx[0], oracle_params(p), record=True)
    compared, excluded = compare_hits(tri.cpu().numpy(), t.cpu().numpy(), orc)
    assert compared >= p.traced() and excluded <= max(3, p.traced() // 10000)


def test_hits_full_lattice_sampled():
    """The bench configuration (urban, 1e7 rays, coherent order, 3 bounces):
    every traced ray is recorded; a random sample is re-traced by the oracle."""
    m = lib()
    w = sg.urban_workload()
    p = params(w)
    tri, t = m.trace_record(ctx(), scene(w.scene), p, w.tx[0])
    tri = tri.cpu().numpy()
    t = t.cpu().numpy()
    assert np.all(tri[0] >= -1)  # every ray traced its first segment
    rng = np.random.default_rng(5)
    pos = np.sort(rng.choice(p.num_rays, size=4000, replace=False))
    for k in range(len(pos) // 1000):
        sub = pos[k * 1000:(k + 1) * 1000]
        # the oracle traces exactly these lattice indices
        orc = sbr.trace(w.scene, w.tx[0], oracle_params(p), record=True, idx=sub)
        compare_hits(tri[:, sub], t[:, sub], orc)


def _coverage_case(name):
    if name == "toy":
        w = sg.toy_workload()
        return w, params(w)
    if name == "urban":
        w = sg.urban_workload(num_rays=400_003)
        return w, params(w)
    if name == "urban_tr38901":
        w = sg.diff_workload(num_rays=300_000)
        return w, params(w)
    if name == "urban_small_grid":  # most rays cannot deposit at the last bounce: they are dropped before it
        w = sg.urban_workload(num_rays=1_000_000)
        w.grid = sg.Grid(37.0, -83.0, 2.0, 45, 35, 2.5)
        return w, params(w)
    if name == "urban_dipole_slant":  # dipole transmitter at -45 degrees, H-pol receive pattern
        w = sg.urban_workload(num_rays=1_000_000)
        w.tx[0].pattern = sg.PATTERN_DIPOLE
        w.tx[0].pol = sg.POL_SLANT_M45
        w.tx[0].pitch = 0.3
        w.rx_ant = sg.Device((0.0, 0.0, 0.0), pattern=sg.PATTERN_ISO, pol=sg.POL_H)
        return w, params(w)
    raise KeyError(name)


@pytest.mark.parametrize("name", ["toy", "urban", "urban_tr38901", "urban_small_grid", "urban_dipole_slant"])
def test_coverage_matches_oracle(name):
    m = lib()
    w, p = _coverage_case(name)
    out = m.coverage_map(ctx(), scene(w.scene), p, w.tx[0], w.grid, rx_ant=w.rx_ant)
    gain = out["gain"].cpu().numpy().astype(np.float64)
    hits = out["hits"].cpu().numpy()
    db = out["gain_db"].cpu().numpy()
    rb = out["ray_bounces"].cpu().numpy()
    g_ref, h_ref, n_amb = sbr.coverage(w.scene, w.tx[0], oracle_params(p), w.grid, rx_ant=w.rx_ant)
    allowed = 2 * (p.max_depth + 1) * n_amb
    # hit counts are integers decided in fp64 on both sides
    assert int((hits != h_ref).sum()) <= allowed
    # every cell with >= 16 hits within 0.1 dB; in fact all agree to fp32 accumulation error
    cmp = (h_ref >= 16) & (hits == h_ref)
    assert cmp.sum() > 50
    ddb = np.abs(10 * np.log10(gain[cmp]) - 10 * np.log10(g_ref[cmp]))
    assert ddb.max() < 0.1
    both = (h_ref > 0) & (hits == h_ref)
    rel = np.abs(gain[both] - g_ref[both]) / g_ref[both]
    assert np.quantile(rel, 0.999) < 1e-4 and int((rel > 1e-3).sum()) <= allowed
    # dB output and empty cells
    assert np.all(np.isneginf(db[hits == 0]))
    assert np.allclose(db[hits > 0], 10 * np.log10(gain[hits > 0]), atol=1e-5)
    # ray-bounce counters: first segment for every ray, then the survivors
    assert rb[0] == p.traced() and np.all(np.diff(rb) <= 0)


@pytest.mark.parametrize("name", ["toy", "urban_stride", "urban_small_grid", "city_stride"])
def test_ray_bounce_counts_match_oracle(name):
    """Rays per depth of a coverage map equal the rays the oracle traces at each
    depth; the last depth's count includes the rays dropped before it because
    their segment cannot cross the coverage plane inside the grid."""
    m = lib()
    if name == "toy":
        w = sg.toy_workload()
        p = params(w)
    elif name == "urban_stride":
        w = sg.urban_workload()
        p = params(w, ray_begin=5, ray_stride=97)
    elif name == "urban_small_grid":
        w, p = _coverage_case(name)
    else:
        w = sg.city_workload(num_rays=100_000_000, blocks=12)
        p = params(w, ray_begin=11, ray_stride=2003)
    out = m.coverage_map(ctx(), scene(w.scene), p, w.tx[0], w.grid)
    rb = out["ray_bounces"].cpu().numpy().astype(np.int64)
    res = sbr.trace(w.scene, w.tx[0], oracle_params(p), record=True)
    ref = np.asarray([int((h != -2).sum()) for h in res.hit_tri], dtype=np.int64)
    amb = int(res.ambiguous.sum())
    assert rb.shape == ref.shape == (p.max_depth + 1,)
    assert rb[0] == ref[0] == p.traced()
    assert np.all(np.abs(rb - ref) <= amb), (rb, ref, amb)


def test_coverage_full_lattice_equals_sum_of_sublattices():
    """Bench configuration (urban, 1e7 rays, depth 3): the full map equals the
    sum of the maps of 10 disjoint sub-lattices (same kernels, different
    launch shapes), up to fp32 atomic ordering."""
    m = lib()
    w = sg.urban_workload()
    p = params(w)
    sc = scene(w.scene)
    full = m.coverage_map(ctx(), sc, p, w.tx[0], w.grid)
    g_full = full["gain"].double()
    h_full = full["hits"].clone()
    g_sum = torch.zeros_like(g_full)
    h_sum = torch.zeros_like(h_full)
    rb = 0
    for b in range(10):
        o = m.coverage_map(ctx(), sc, params(w, ray_begin=b, ray_stride=10), w.tx[0], w.grid)
        g_sum += o["gain"].double()
        h_sum += o["hits"]
        rb += int(o["ray_bounces"].sum())
    assert torch.equal(h_full, h_sum)
    assert rb == int(full["ray_bounces"].sum())
    nz = h_full > 0
    rel = ((g_full - g_sum).abs() / g_sum.clamp_min(1e-30))[nz]
    assert float(rel.max()) < 1e-4
    assert int(h_full.sum()) > 1_000_000


def test_city_coverage_full_equals_sum_of_sublattices():
    """Large city at its full size (about 220k triangles, 1e8 rays, 5 bounces,
    2000x2000 cells): the map equals the sum of the maps of 4 disjoint
    sub-lattices (hit counts exactly, gains to fp32 atomic ordering)."""
    m = lib()
    w = sg.city_workload()
    p = params(w)
    sc = scene(w.scene)
    assert sc.info()["num_triangles"] > 200_000
    full = m.coverage_map(ctx(), sc, p, w.tx[0], w.grid)
    g_full = full["gain"].double()
    h_full = full["hits"].clone()
    rb_full = int(full["ray_bounces"].sum())
    g_sum = torch.zeros_like(g_full)
    h_sum = torch.zeros_like(h_full)
    rb = 0
    for b in range(4):
        o = m.coverage_map(ctx(), sc, params(w, ray_begin=b, ray_stride=4), w.tx[0], w.grid)
        g_sum += o["gain"].double()
        h_sum += o["hits"]
        rb += int(o["ray_bounces"].sum())
    assert torch.equal(h_full, h_sum)
    assert rb == rb_full and rb > 100_000_000
    nz = h_full > 0
    rel = ((g_full - g_sum).abs() / g_sum.clamp_min(1e-30))[nz]
    assert float(rel.max()) < 1e-4
    assert int(nz.sum()) > 100_000


def test_argument_errors_are_reported():
    m = lib()
    from paper_2303_11103_amd._lib import RTError
    w = sg.toy_workload()
    sc = scene(w.scene)
    with pytest.raises(RTError, match="max_depth"):
        m.coverage_map(ctx(), sc, params(w, max_depth=9), w.tx[0], w.grid)
    with pytest.raises(RTError, match="ray_stride"):
        m.coverage_map(ctx(), sc, params(w, ray_stride=0), w.tx[0], w.grid)
    bad = sg.Device((float("nan"), 0.0, 10.0))
    with pytest.raises(RTError, match="non-finite"):
        m.coverage_map(ctx(), sc, params(w), bad, w.grid)
    with pytest.raises(RTError, match="vertex index"):
        F = w.scene.F.copy()
        F[0, 0] = 10_000
        m.Scene(ctx(), w.scene.V, F, w.scene.tri_mat, w.scene.materials)


def test_coverage_maps_of_several_transmitters_equal_single_calls():
    m = lib()
    w = sg.urban_workload(num_rays=300_000)
    p = params(w)
    sc = scene(w.scene)
    pos = sg.rooftop_tx_positions(w.scene, 3, seed=4)
    txs = [sg.Device(tuple(float(x) for x in q)) for q in pos]
    many = m.coverage_maps(ctx(), sc, p, txs, w.grid, want_db=True)
    for k, tx in enumerate(txs):
        one = m.coverage_map(ctx(), sc, p, tx, w.grid)
        assert torch.equal(many["hits"][k], one["hits"])
        assert torch.allclose(many["gain"][k].double(), one["gain"].double(), rtol=1e-6, atol=0.0)
        assert torch.allclose(many["gain_db"][k][one["hits"] > 0], one["gain_db"][one["hits"] > 0], atol=1e-5)
    with pytest.raises(RuntimeError, match="at least one transmitter"):
        m.coverage_maps(ctx(), sc, p, [], w.grid)
