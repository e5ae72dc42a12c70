#!/usr/bin/env python3
"""Benchmark of the ray tracer's hot path on one MI355X.

Workload (timed step): the coverage map of the urban-canyon scene -- 8x8 box
buildings (770 triangles, concrete/glass at 3.5 GHz), one isotropic V-pol
transmitter 2 m above a roof corner, 1e7 Fibonacci-lattice rays, up to 3
specular reflections, 400x400 cells of 1 m at 1.5 m height.  One step =
Fibonacci ray generation, closest-hit BVH traversal, coverage deposit,
Fresnel reflection and queue compaction for every bounce, then the dB map.

Prints one JSON line: value = ray-bounces (closest-hit queries, counted on
the device) per second; roofline of the depth-0 shoot-and-bounce launch
(algorithmic FLOPs from counted BVH node visits and triangle tests, divided
by its HIP-event duration on the library's stream; all launches reported
beside it); the FP64 CPU oracle timed on a
bounded ray sample of the same workload; and side measurements of the paths
(image method) and gradient kernels.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BJ_METRIC = "M ray-bounces/s + coverage-map ms vs oracle; surrogate maps/s at <=3 dB RMSE"
# Algorithmic work per unit (floating-point operations the method needs; an
# FMA counts 2, an add/mul/min/max/compare 1):
#   BVH inner-node visit = four fp32 ray/box slab tests (the children of a
#     4-wide node): 24 FMA + 48 min/max + 12 for the interval tests = 108;
#   triangle test = fp64 Moller-Trumbore without division: 46;
#   every traced segment: coverage-plane crossing, cell index, receive
#     pattern and |F_rx . E|^2 deposit: 40;
#   every surviving ray (reflection): Fresnel r_perp/r_par (complex sqrt and
#     two complex divisions), perpendicular/parallel bases, reflected
#     direction and hit point, 3-vector complex field update: 160;
#   every ray at depth 0: Fibonacci direction (z, rho, sincos of the golden
#     phase) and transmit pattern: 70.
FLOP_NODE = 108.0
FLOP_TRI = 46.0
FLOP_DEPOSIT = 40.0
FLOP_REFLECT = 160.0
FLOP_RAYGEN = 70.0
# MI355X VALU: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s,
# FMA = 2 flops -> 78.6 TFLOP/s for fp64 and for non-packed fp32 (the build
# disables packed fp32).
PEAK_ALU_TFLOPS = 78.6
PEAK_LANE_OPS = 39.3e12
# Lane operations (one per issued lane instruction, an FMA counts once) of the
# traversal terms, exact for the code: a 4-wide node visit is 4 x (6 FMA + 12
# min/max + 3) = 84; a Moller-Trumbore test is 32 (two cross products 6 each,
# four dot products 3 each, 3 subtractions, 5 comparisons).  The other terms
# (deposit, reflection, ray generation) are left out, so the lane-op fraction
# below is a lower bound.
LANE_NODE = 84.0
LANE_TRI = 32.0
COPY_PROBE_BYTES = 256 << 20
# Sources that make up the shoot-and-bounce kernel: HBM traffic measured with
# counters is reported only while they are unchanged.
KERNEL_SOURCES = ["paper_2303_11103_amd/csrc/" + f for f in
                  ("trace.hip", "traverse.h", "device.h", "kernels.h", "layout.h", "api.hip", "scene.cpp")]
TRAFFIC_PROFILE = "profiles/sbr_bounce_urban_hbm_traffic.md"


def kernel_sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_per_launch():
    """HBM bytes per depth-0 launch from the committed counter profile (FETCH_SIZE
    + WRITE_SIZE, scaled by the copy probe), or None when the profile is missing
    or was taken on other kernel sources."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("traffic:"):
            for kv in line[len("traffic:"):].split():
                k, v = kv.split("=")
                vals[k] = v
    if vals.get("sources") != kernel_sources_digest() or "bytes_per_launch" not in vals:
        return None
    return float(vals["bytes_per_launch"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(seconds_budget: float = 20.0):
    """Time the FP64 oracle on a strided sample of the same workload."""
    import numpy as np
    import scenegen as sg
    from oracle import native, sbr
    w = sg.urban_workload()
    threads = native.default_threads()
    stride = 1000
    # grow the sample until it takes about seconds_budget (bounded: at most all rays)
    while True:
        p = sbr.TraceParams(num_rays=w.num_rays, max_depth=w.max_depth, ray_begin=0, ray_stride=stride)
        t0 = time.perf_counter()
        r = sbr.trace(w.scene, w.tx[0], p, grid=w.grid, record=True, threads=threads)
        dt = time.perf_counter() - t0
        segs = int(sum(int((h != -2).sum()) for h in r.hit_tri))
        if dt > seconds_budget / 3 or stride == 1:
            break
        stride = max(1, int(stride * dt / seconds_budget))
    return {"value": segs / dt / 1e6, "unit": "M ray-bounces/s", "cores": threads, "kind": "oracle",
            "sample": "urban canyon coverage map, lattice rays 0, %d, 2*%d, ... of 1e7 (%d rays, %d ray-bounces, "
                      "depth 3), %.1f s on %d threads" % (stride, stride, len(r.ray_idx), segs, dt, threads)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the paths/gradient side measurements")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the learned-surrogate measurement")
    ap.add_argument("--surrogate-steps", type=int, default=20000)
    ap.add_argument("--surrogate-tx", type=int, default=4096,
                    help="training maps of the surrogate (plus 1/16 as many validation and test maps each)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed region, copy %d MiB once (reference kernel for HBM counters)" % (
                        256))
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the shoot-and-bounce workload of one transmitter runs on a single "
              "MI355X (rays would shard by lattice range, maps reduce with one all-reduce); got --gpus %d" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import ctypes

    import numpy as np
    import torch

    import paper_2303_11103_amd as rt
    from paper_2303_11103_amd._lib import check, lib
    import scenegen as sg

    dev = torch.device("cuda", 0)
    w = sg.urban_workload()
    ctx = rt.Context(0)
    scene = rt.Scene.from_scenegen(ctx, w.scene)
    info = scene.info()
    p = rt.TraceParams(w.scene.freq_hz, w.max_depth, w.num_rays)
    tx = w.tx[0]
    out = {"gain": torch.empty((w.grid.ny, w.grid.nx), dtype=torch.float32, device=dev),
           "hits": torch.empty((w.grid.ny, w.grid.nx), dtype=torch.int32, device=dev),
           "gain_db": torch.empty((w.grid.ny, w.grid.nx), dtype=torch.float32, device=dev),
           "ray_bounces": torch.empty(w.max_depth + 1, dtype=torch.int64, device=dev)}
    log("bench: urban canyon, %d rays, depth %d, BVH %d nodes (build %.1f ms)" % (
        w.num_rays, w.max_depth, info["bvh_nodes"], info["build_ms"]))
    for _ in range(args.warmup):
        rt.coverage_map(ctx, scene, p, tx, w.grid, out=out)
    torch.cuda.synchronize()
    log("bench: warmup done")

    nd = w.max_depth + 1
    check(lib.rt_profile_enable(ctx.h, 1))
    stream = torch.cuda.current_stream(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        rt.coverage_map(ctx, scene, p, tx, w.grid, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    check(lib.rt_profile_enable(ctx.h, 0))
    launches = (ctypes.c_int64 * nd)()
    kms = (ctypes.c_double * nd)()
    check(lib.rt_profile_read(ctx.h, nd, launches, kms))
    ms_step = (t1 - t0) * 1e3 / args.steps
    ms_step_ev = ev0.elapsed_time(ev1) / args.steps
    rb_depth = out["ray_bounces"].cpu().numpy().astype(np.int64)
    ray_bounces = int(rb_depth.sum())
    value = ray_bounces / (ms_step / 1e3) / 1e6
    log("bench: %.3f ms/step (events %.3f), %d ray-bounces/step -> %.1f M ray-bounces/s" % (
        ms_step, ms_step_ev, ray_bounces, value))

    # work counters (one extra, untimed run with per-ray counters)
    work = torch.zeros(3 * nd, dtype=torch.int64, device=dev)
    g2 = torch.empty_like(out["gain"])
    h2 = torch.empty_like(out["hits"])
    pc, tc, rc, gc = p.c(), rt.rt.device_struct(tx), rt.rt.device_struct(w.rx_ant), rt.rt.grid_struct(w.grid)
    ctx._bind_stream()
    check(lib.rt_coverage_work(ctx.h, scene.h, ctypes.byref(pc), ctypes.byref(tc), ctypes.byref(rc),
                               ctypes.byref(gc), ctypes.c_void_p(g2.data_ptr()), ctypes.c_void_p(h2.data_ptr()),
                               ctypes.c_void_p(work.data_ptr())))
    wk = work.cpu().numpy().reshape(3, nd)
    assert np.array_equal(wk[0], rb_depth), (wk[0], rb_depth)
    survivors = np.append(wk[0][1:], 0)
    flops_depth = FLOP_NODE * wk[1] + FLOP_TRI * wk[2] + FLOP_DEPOSIT * wk[0] + FLOP_REFLECT * survivors
    flops_depth[0] += FLOP_RAYGEN * wk[0][0]
    k_ms = np.asarray(list(kms)) / np.maximum(1, np.asarray(list(launches)))  # per launch, per depth
    per_step_kernel_ms = float(k_ms.sum())
    achieved_all = flops_depth.sum() / (per_step_kernel_ms / 1e3) / 1e12
    # dominant kernel: the depth-0 launch (sbr_bounce<1, true>: ray generation,
    # first closest hit, deposit, reflection), the longest single launch of a step
    dom = int(np.argmax(k_ms))
    achieved = flops_depth[0] / (k_ms[0] / 1e3) / 1e12
    roofline = {
        "bound": "alu",
        "achieved": round(float(achieved), 3),
        "peak": PEAK_ALU_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(float(achieved / PEAK_ALU_TFLOPS), 4),
        "traffic": traffic_per_launch(),
        "kernel": "sbr_bounce<coverage, first bounce> (depth-0 launch: %d rays)" % int(wk[0][0]),
        "kernel_ms": round(float(k_ms[0]), 4),
        "flop_per_launch": float(flops_depth[0]),
        "traversal_lane_op_frac": round(float((LANE_NODE * wk[1][0] + LANE_TRI * wk[2][0]) / (k_ms[0] / 1e3)
                                              / PEAK_LANE_OPS), 4),
        "longest_launch": "depth %d, %.3f ms" % (dom, float(k_ms[dom])),
        "all_launches": {"kernel_ms_per_depth": [round(float(x), 4) for x in k_ms],
                         "achieved": round(float(achieved_all), 3),
                         "frac": round(float(achieved_all / PEAK_ALU_TFLOPS), 4)},
        "node_visits_per_ray_bounce": round(float(wk[1].sum() / wk[0].sum()), 2),
        "tri_tests_per_ray_bounce": round(float(wk[2].sum() / wk[0].sum()), 2),
        "flop_per_ray_bounce": round(float(flops_depth.sum() / wk[0].sum()), 1),
        "rays_per_depth": [int(x) for x in wk[0]],
        "node_visits_per_depth": [int(x) for x in wk[1]],
        "tri_tests_per_depth": [int(x) for x in wk[2]],
    }
    log("bench: depth-0 launch %.4f ms, %.2f TFLOP/s algorithmic (%.1f%% of %.1f); all launches %.3f ms/step, "
        "%.2f TFLOP/s" % (k_ms[0], achieved, 100 * achieved / PEAK_ALU_TFLOPS, PEAK_ALU_TFLOPS,
                          per_step_kernel_ms, achieved_all))
    if args.copy_probe:
        # a plain device copy of known size: the HBM counters of the profile runs
        # are scaled by what they read for it
        src = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    result = {
        "metric": BJ_METRIC,
        "value": round(value, 2),
        "unit": "M ray-bounces/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 geometry + f32 field",
        "data": "synthetic",
        "config": {"workload": "urban canyon coverage map: 8x8 boxes (770 tris), 1e7 rays, depth 3, "
                               "400x400 cells of 1 m, 3.5 GHz",
                   "num_rays": w.num_rays, "max_depth": w.max_depth, "grid": [w.grid.ny, w.grid.nx],
                   "triangles": int(w.scene.nt)},
        "coverage_map_ms": round(ms_step, 4),
        "ray_bounces_per_step": ray_bounces,
        "roofline": roofline,
    }

    if not args.no_extras:
        try:
            result.update(extras(rt, ctx, scene, w, torch))
        except Exception as e:  # side measurements must not hide the main line
            log("bench: extras failed: %r" % (e,))
            result["extras_error"] = repr(e)

    if not args.no_surrogate:
        try:
            result["surrogate"] = surrogate_bench(rt, ctx, scene, w, torch, steps=args.surrogate_steps,
                                                  n_train=args.surrogate_tx)
        except Exception as e:
            log("bench: surrogate failed: %r" % (e,))
            result["surrogate_error"] = repr(e)

    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on a ray sample ...")
        cb = cpu_baseline()
        cb["vs_gpu"] = round(value / cb["value"], 1)
        result["cpu_baseline"] = cb
    print(json.dumps(result), flush=True)


def extras(rt, ctx, scene, w, torch):
    """Paths for the workload's 16 receivers and the power gradient (timed)."""
    import scenegen as sg
    res = {}
    p = rt.TraceParams(w.scene.freq_hz, w.max_depth, w.num_rays, max_paths_per_rx=64)
    rt.compute_paths(ctx, scene, p, w.tx, w.rx)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    o = rt.compute_paths(ctx, scene, p, w.tx, w.rx)
    torch.cuda.synchronize()
    res["paths_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
    res["paths_found"] = int(o["num_paths"].sum())
    res["path_candidates"] = rt.last_candidate_count(ctx)
    d = sg.diff_workload()
    pd = rt.TraceParams(d.scene.freq_hz, d.max_depth, d.num_rays, max_paths_per_rx=64)
    sd = scene if d.scene.digest() == w.scene.digest() else rt.Scene.from_scenegen(ctx, d.scene)
    od = rt.compute_paths(ctx, sd, pd, d.tx, d.rx)
    torch.cuda.synchronize()
    dL = torch.ones(len(d.rx), dtype=torch.float64, device=ctx.torch_device)
    rt.paths_power_grad(ctx, sd, pd, d.tx[0], d.rx, od["depth"][0], od["faces"][0], dL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        rt.paths_power_grad(ctx, sd, pd, d.tx[0], d.rx, od["depth"][0], od["faces"][0], dL)
    torch.cuda.synchronize()
    res["grad_ms"] = round((time.perf_counter() - t0) * 1e3 / 10, 4)
    res["grad_paths"] = int((od["depth"][0] >= 0).sum())
    # coverage-map gradient (materials, tx yaw and pitch) of the whole map at
    # the workload's lattice: record the hits, then replay with field tangents
    pg = rt.TraceParams(d.scene.freq_hz, w.max_depth, w.num_rays)
    tri, tt = rt.trace_record(ctx, sd, pg, d.tx[0])
    rt.coverage_grad(ctx, sd, pg, d.tx[0], w.grid, tri, tt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        tri, tt = rt.trace_record(ctx, sd, pg, d.tx[0])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(3):
        og = rt.coverage_grad(ctx, sd, pg, d.tx[0], w.grid, tri, tt)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    segs = int((tri != -2).sum())
    res["coverage_grad"] = {"workload": "urban coverage map, 1e7 rays, depth 3, 400x400 cells; d/d(eps_r, sigma) "
                                        "of 2 materials, tx yaw, pitch",
                            "record_ms": round((t1 - t0) * 1e3 / 3, 3), "replay_ms": round((t2 - t1) * 1e3 / 3, 3),
                            "segments": segs, "M_segments_per_s": round(segs / ((t2 - t1) / 3) / 1e6, 1),
                            "region_gain": float(og[0])}
    log("bench: coverage grad %s" % res["coverage_grad"])
    # channel frequency responses (128 subcarriers, 30 kHz) of the 256 receivers
    # of the differentiation case, their adjoint and the material gradient
    od = rt.compute_paths(ctx, sd, pd, d.tx, d.rx)
    kw = dict(num_subcarriers=128, spacing=30e3)
    H = rt.paths_cfr(ctx, od, pd.freq_hz, **kw)
    G = torch.ones_like(H)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        H = rt.paths_cfr(ctx, od, pd.freq_hz, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(10):
        g = rt.paths_cfr_adjoint(ctx, od, G, pd.freq_hz, **kw)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(10):
        rt.paths_coef_grad(ctx, sd, pd, d.tx[0], d.rx, od["depth"][0], od["faces"][0], g[0])
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    res["cfr"] = {"workload": "256 rx of the differentiation case, %d paths, 128 subcarriers" %
                              int((od["depth"] >= 0).sum()),
                  "cfr_ms": round((t1 - t0) * 1e2, 4), "adjoint_ms": round((t2 - t1) * 1e2, 4),
                  "coef_grad_ms": round((t3 - t2) * 1e2, 4)}
    log("bench: cfr %s" % res["cfr"])
    # the urban map with diffuse scattering (S = 0.6 concrete, 0.35 glass)
    ss = rt.Scene.from_scenegen(ctx, w.scene)
    ss.set_scattering([0.6, 0.35], 11)
    outs = rt.coverage_map(ctx, ss, rt.TraceParams(w.scene.freq_hz, w.max_depth, w.num_rays), w.tx[0], w.grid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        outs = rt.coverage_map(ctx, ss, rt.TraceParams(w.scene.freq_hz, w.max_depth, w.num_rays), w.tx[0], w.grid)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / 5
    rbs = int(outs["ray_bounces"].sum())
    res["scattering"] = {"workload": "urban coverage map with Lambertian scattering S = (0.6, 0.35), 1e7 rays, depth 3",
                         "coverage_map_ms": round(ms, 3), "ray_bounces": rbs,
                         "M_ray_bounces_per_s": round(rbs / (ms / 1e3) / 1e6, 1)}
    log("bench: scattering %s" % res["scattering"])
    ss.close()
    # large procedural city: coverage map at full size
    c = sg.city_workload()
    t0 = time.perf_counter()
    sc = rt.Scene.from_scenegen(ctx, c.scene)
    scene_s = time.perf_counter() - t0
    pc = rt.TraceParams(c.scene.freq_hz, c.max_depth, c.num_rays)
    dev = ctx.torch_device
    outc = {"gain": torch.empty((c.grid.ny, c.grid.nx), dtype=torch.float32, device=dev),
            "hits": torch.empty((c.grid.ny, c.grid.nx), dtype=torch.int32, device=dev),
            "gain_db": torch.empty((c.grid.ny, c.grid.nx), dtype=torch.float32, device=dev),
            "ray_bounces": torch.empty(c.max_depth + 1, dtype=torch.int64, device=dev)}
    rt.coverage_map(ctx, sc, pc, c.tx[0], c.grid, out=outc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2):
        rt.coverage_map(ctx, sc, pc, c.tx[0], c.grid, out=outc)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / 2
    rbc = int(outc["ray_bounces"].sum())
    info = sc.info()
    res["city"] = {"workload": "large city coverage map: 50x50 blocks (%d tris), 1e8 rays, depth 5, 2000x2000 "
                               "cells of 1 m, 28 GHz, TR 38.901 tx" % info["num_triangles"],
                   "coverage_map_ms": round(ms, 3), "ray_bounces": rbc,
                   "M_ray_bounces_per_s": round(rbc / (ms / 1e3) / 1e6, 1),
                   "bvh_nodes": info["bvh_nodes"], "bvh_build_ms": round(info["build_ms"], 1),
                   "scene_create_s": round(scene_s, 2)}
    # paths to the 4096 street receivers with reception-sphere candidates
    pp = rt.TraceParams(c.scene.freq_hz, c.max_depth, c.num_rays, max_paths_per_rx=256, cand_mode=1,
                        sphere_kappa=2.0)
    t0 = time.perf_counter()
    op = rt.compute_paths(ctx, sc, pp, c.tx, c.rx)
    torch.cuda.synchronize()
    res["city"]["paths_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    res["city"]["paths_found"] = int(op["num_paths"].sum())
    res["city"]["rx_with_paths"] = int((op["num_paths"] > 0).sum())
    res["city"]["sphere_pairs"] = rt.last_candidate_count(ctx)
    log("bench: city %s" % res["city"])
    sc.close()
    return res


def surrogate_bench(rt, ctx, scene, w, torch, steps=20000, n_train=4096, seed=3):
    """Learned surrogate on the urban scene: ray-traced maps (1e7 rays, depth 3,
    200x200 cells of 2 m) for transmitters uniform over the rooftops, n_train
    training maps plus n_train/16 validation and n_train/16 test maps; trained with the library's MFMA
    kernels; reports test RMSE in dB over cells with >= 16 hits, the
    fallback mask (cells whose validation RMSE exceeds 6 dB) and maps/s of
    the surrogate and of the ray tracer at the same resolution."""
    import numpy as np
    import scenegen as sg
    from paper_2303_11103_amd import surrogate as S
    grid = sg.Grid(-200.0, -200.0, 2.0, 200, 200, 1.5)
    n_val = n_test = max(1, n_train // 16)
    n_tx = n_train + n_val + n_test
    tx_np = sg.rooftop_tx_positions(w.scene, n_tx, seed=seed)
    dev = ctx.torch_device
    tx = torch.tensor(tx_np, device=dev)
    p = rt.TraceParams(w.scene.freq_hz, 3, 10_000_000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    maps, mask = S.ray_traced_maps(ctx, scene, p, tx_np, grid)
    torch.cuda.synchronize()
    rt_s = time.perf_counter() - t0
    n_tr = n_train
    tr, va, te = slice(0, n_tr), slice(n_tr, n_tr + n_val), slice(n_tr + n_val, n_tx)
    # targets: cells with >= 16 hits; the dB values there are finite
    maps = torch.where(mask.bool(), maps, torch.zeros_like(maps))
    lo = np.array([-200.0, -200.0, 10.0, -200.0, -200.0])
    hi = np.array([200.0, 200.0, 65.0, 200.0, 200.0])
    # Fourier rows: 8 on the transmitter (low frequencies), 16 on the cell, 40 on the
    # cell relative to the transmitter; the network learns the residual over the
    # free-space gain of each link
    m = S.MLP(ctx, batch=32768, ff_scale=1.0, ff_scale_cell=4.0, seed=seed, center=(lo + hi) / 2, half=(hi - lo) / 2,
              prior=(w.scene.freq_hz, grid.z), ff_rows_tx=8, ff_rows_rel=40, ff_scale_rel=32.0)
    rep = S.train(m, maps[tr].contiguous(), mask[tr].contiguous(), tx[tr].contiguous(), grid, steps=steps, lr=2e-3,
                  seed=seed)
    pv = m.predict_maps(tx[va], grid)
    fb = S.fallback_mask(pv, maps[va], mask[va], threshold_db=6.0)
    val_rmse = S.rmse_db(pv, maps[va], mask[va])
    pt = m.predict_maps(tx[te], grid)
    test_rmse = S.rmse_db(pt, maps[te], mask[te])
    keep = mask[te].bool() & ~fb[None]
    d = (pt - maps[te])[keep]
    test_rmse_nofb = float(torch.sqrt(torch.mean(d * d))) if d.numel() else float("nan")
    # inference speed: 1024 transmitters per call
    q = tx[:1024].contiguous() if n_tx >= 1024 else tx
    out = torch.empty((q.shape[0], grid.ny, grid.nx), dtype=torch.float32, device=dev)
    m.predict_maps(q, grid, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.predict_maps(q, grid, out=out)
    torch.cuda.synchronize()
    inf_s = time.perf_counter() - t0
    sur_maps_s = q.shape[0] / inf_s
    rt_maps_s = n_tx / rt_s
    fb_frac = float(fb.float().mean())
    res = {
        "maps_per_s": round(sur_maps_s, 1),
        "ray_tracer_maps_per_s": round(rt_maps_s, 1),
        "speedup": round(sur_maps_s / rt_maps_s, 1),
        "test_rmse_db": round(test_rmse, 3),
        "test_rmse_db_outside_fallback": round(test_rmse_nofb, 3),
        "val_rmse_db": round(val_rmse, 3),
        "fallback_cell_fraction": round(fb_frac, 4),
        # with a non-empty fallback mask every full-map query also runs the ray tracer
        "maps_per_s_with_fallback": round(sur_maps_s if fb_frac == 0 else 1.0 / (1.0 / sur_maps_s + 1.0 / rt_maps_s), 1),
        "train_steps": rep.steps, "train_s": round(rep.seconds, 1), "train_final_loss": round(rep.final_loss, 3),
        "dataset": "%d tx (%d train / %d val / %d test), 200x200 cells of 2 m, 1e7 rays, depth 3" % (
            n_tx, n_tr, n_val, n_test),
    }
    log("bench: surrogate %s" % res)
    m.close()
    return res


if __name__ == "__main__":
    main()
