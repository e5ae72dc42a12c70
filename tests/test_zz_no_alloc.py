"""The allocation-free coverage entry point (rt_coverage_map_noalloc) against
rt_coverage_map on the same inputs, called through the C ABI: two calls in a
row, the second on a smaller input, so that the fixed scratch array is reused
with different sizes and must be cleared between calls."""
import ctypes

import numpy as np
import pytest
import torch

import scenegen as sg
from gpu_common import ctx, lib, params, requires_gpu, scene

pytestmark = [pytest.mark.gpu, requires_gpu]


def _run(entry, c, s, p, tx, grid):
    m = lib()
    from paper_2303_11103_amd import _lib as L
    from paper_2303_11103_amd import rt as R
    dev = c.torch_device
    out = {"gain": torch.full((grid.ny, grid.nx), 7.0, dtype=torch.float32, device=dev),
           "hits": torch.full((grid.ny, grid.nx), 7, dtype=torch.int32, device=dev),
           "gain_db": torch.empty((grid.ny, grid.nx), dtype=torch.float32, device=dev),
           "ray_bounces": torch.full((p.max_depth + 1,), 7, dtype=torch.int64, device=dev)}
    rx = R.device_struct(sg.Device((0.0, 0.0, 0.0)))
    c._bind_stream()
    pc, tc, gc = p.c(), R.device_struct(tx), R.grid_struct(grid)
    L.check(getattr(L.lib, entry)(c.h, s.h, ctypes.byref(pc), ctypes.byref(tc), ctypes.byref(rx), ctypes.byref(gc),
                                  ctypes.c_void_p(out["gain"].data_ptr()), ctypes.c_void_p(out["hits"].data_ptr()),
                                  ctypes.c_void_p(out["gain_db"].data_ptr()),
                                  ctypes.c_void_p(out["ray_bounces"].data_ptr())))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same(a, b):
    # integer outputs bit-exact; the fp32 gain sums differ only in the order of
    # their atomic additions (chunks of 2^19 rays here, 2^27 in rt_coverage_map)
    assert np.array_equal(a["hits"], b["hits"])
    assert np.array_equal(a["ray_bounces"], b["ray_bounces"])
    hit = b["hits"] > 0
    assert np.array_equal(a["gain"] > 0, b["gain"] > 0)
    rel = np.abs(a["gain"][hit] - b["gain"][hit]) / b["gain"][hit]
    assert rel.max() < 1e-4, rel.max()
    assert np.all(a["gain"][~hit] == 0.0)
    ddb = np.abs(a["gain_db"][hit] - b["gain_db"][hit])
    assert ddb.max() < 1e-3
    assert np.all(np.isneginf(a["gain_db"][~hit]))


def test_noalloc_coverage_equals_coverage_map_twice():
    c = ctx()
    # first call: urban canyon, 2.5e6 rays (five chunks of the fixed queues), depth 3
    w = sg.urban_workload()
    s = scene(w.scene)
    p = params(w, num_rays=2_500_000)
    a = _run("rt_coverage_map_noalloc", c, s, p, w.tx[0], w.grid)
    b = _run("rt_coverage_map", c, s, p, w.tx[0], w.grid)
    print("urban: %d hit cells, %d ray-bounces" % (int((b["hits"] > 0).sum()), int(b["ray_bounces"].sum())),
          flush=True)
    _same(a, b)
    # second call, smaller: the toy scene, 1e5 rays, depth 1, 200 x 200 cells
    t = sg.toy_workload()
    st = scene(t.scene)
    pt = params(t)
    a2 = _run("rt_coverage_map_noalloc", c, st, pt, t.tx[0], t.grid)
    b2 = _run("rt_coverage_map", c, st, pt, t.tx[0], t.grid)
    _same(a2, b2)
    assert int(a2["ray_bounces"].sum()) < int(a["ray_bounces"].sum())


def test_noalloc_rejects_bad_arguments_like_coverage_map():
    from paper_2303_11103_amd import _lib as L
    from paper_2303_11103_amd import rt as R
    c = ctx()
    t = sg.toy_workload()
    st = scene(t.scene)
    p = params(t, max_depth=9)
    pc, tc, gc = p.c(), R.device_struct(t.tx[0]), R.grid_struct(t.grid)
    rx = R.device_struct(sg.Device((0.0, 0.0, 0.0)))
    g = torch.empty((t.grid.ny, t.grid.nx), dtype=torch.float32, device=c.torch_device)
    h = torch.empty((t.grid.ny, t.grid.nx), dtype=torch.int32, device=c.torch_device)
    rc = L.lib.rt_coverage_map_noalloc(c.h, st.h, ctypes.byref(pc), ctypes.byref(tc), ctypes.byref(rx),
                                       ctypes.byref(gc), ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(h.data_ptr()),
                                       None, None)
    assert rc == L.RT_ERR_ARG
