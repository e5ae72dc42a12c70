"""Shared helpers of the GPU parity tests (imported by tests only)."""
import numpy as np
import pytest
import torch

import scenegen as sg
from oracle import geom, sbr

requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")


def lib():
    import paper_2303_11103_amd as m  # raises if the HIP library is missing
    return m


_CTX = {}


def ctx():
    m = lib()
    if "ctx" not in _CTX:
        _CTX["ctx"] = m.Context(0)
    return _CTX["ctx"]


def scene(s):
    m = lib()
    key = ("scene", s.name, s.digest())
    if key not in _CTX:
        _CTX[key] = m.Scene.from_scenegen(ctx(), s)
    return _CTX[key]


def params(w, **kw):
    m = lib()
    p = dict(freq_hz=w.scene.freq_hz, max_depth=w.max_depth, num_rays=w.num_rays)
    p.update(kw)
    return m.TraceParams(**p)


def oracle_params(p):
    return sbr.TraceParams(num_rays=p.num_rays, max_depth=p.max_depth, tmin=p.t_min, ray_begin=p.ray_begin,
                           ray_stride=p.ray_stride)


def compare_hits(gpu_tri, gpu_t, orc, delta=1e-6):
    """Per bounce, triangle ids must be identical for every ray that has not
    passed within delta of an edge (or a coincident-triangle tie) so far;
    returns (compared ray-bounces, excluded rays)."""
    D1 = len(orc.hit_tri)
    n = orc.hit_tri[0].shape[0]
    ok_ray = np.ones(n, dtype=bool)
    compared = 0
    for k in range(D1):
        o_tri = orc.hit_tri[k]
        sel = ok_ray & (o_tri != -2)
        amb = orc.margin[k] < delta
        cmp = sel & ~amb
        g = gpu_tri[k]
        bad = np.nonzero(cmp & (g != o_tri))[0]
        assert bad.size == 0, "bounce %d: %d mismatches, first rays %s gpu %s oracle %s" % (
            k, bad.size, bad[:5], g[bad[:5]], o_tri[bad[:5]])
        hit = cmp & (o_tri >= 0)
        if hit.any():
            rel = np.abs(gpu_t[k][hit] - orc.hit_t[k][hit]) / (1.0 + orc.hit_t[k][hit])
            assert rel.max() < 1e-9, rel.max()
        # rays terminated by the oracle must be terminated on the GPU too
        dead = cmp & (o_tri == -1)
        assert np.all(g[dead] == -1)
        compared += int(cmp.sum())
        ok_ray &= ~amb
    return compared, int((~ok_ray).sum())
