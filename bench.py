#!/usr/bin/env python3
"""Benchmark of the ray tracer's hot path on one MI355X.

Headline workload (timed step): the coverage map of the large procedural
city -- 50x50 blocks of extruded convex polygons (about 220k triangles,
concrete/glass/metal at 28 GHz), a TR 38.901 transmitter (pitch +10 deg) 2 m
above the tallest roof near the centre, 1e8 Fibonacci-lattice rays, up to 5
specular reflections, 2000x2000 cells of 1 m at 1.5 m height.  One step =
ray generation, closest-hit BVH traversal, coverage deposit, Fresnel
reflection and queue compaction for every bounce (one chunk of 1e8 rays),
then the dB map.  The urban canyon (8x8 boxes, 1e7 rays, depth 3, 400x400
cells) is measured the same way as a secondary object.

Prints one JSON line: value = ray-bounces (closest-hit queries, counted on
the device) per second over the timed steps; the roofline of the
shoot-and-bounce kernel with the largest share of the step time, from the
work the method needs per unit (12 flop per child-box slab test, 46 per
Moller-Trumbore test, 325 per ray-bounce for shading, crossing and deposit),
with the units counted on the device, divided by that kernel's HIP-event
durations on the library's stream; the FP64 CPU oracle timed on a strided
lattice sample of the same workload (its rate per ray-bounce extrapolates to
the full map); and side measurements (paths, gradients, channel responses,
scattering, learned surrogate).

    python bench.py [--gpus 1] [--steps 10] [--warmup 3] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BJ_METRIC = "M ray-bounces/s + coverage-map ms vs oracle; surrogate maps/s at <=3 dB RMSE"
# Algorithmic work per unit (floating-point operations the method needs; an
# FMA counts 2, min/max and compares are not counted):
#   child-box slab test with a precomputed inverse direction: 6 FMA = 12;
#   fp64 Moller-Trumbore test (two cross products, four dot products, one
#     division): 46;
#   every ray-bounce: reflection (complex square root, two complex divisions,
#     perpendicular/parallel bases, reflected direction, 3-vector complex field
#     update, about 300) plus plane crossing and cell deposit (about 25): 325.
FLOP_BOX = 12.0
FLOP_TRI = 46.0
FLOP_RAY_BOUNCE = 325.0
# MI355X VALU: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s,
# FMA = 2 flops -> 78.6 TFLOP/s for fp64 and for non-packed fp32 (the build
# disables packed fp32).
PEAK_ALU_TFLOPS = 78.6
COPY_PROBE_BYTES = 256 << 20
# Sources that make up the shoot-and-bounce kernels: HBM traffic measured with
# counters is reported only while they are unchanged.
KERNEL_SOURCES = ["paper_2303_11103_amd/csrc/" + f for f in
                  ("trace.hip", "traverse.h", "device.h", "kernels.h", "layout.h", "api.hip", "scene.cpp")]
TRAFFIC_PROFILE = "profiles/sbr_bounce_hbm_traffic.md"
KERNEL_KIND = {"first": "sbr_bounce<coverage> depth-0 launch (ray generation + first bounce)",
               "bounce": "sbr_bounce<coverage> depth >= 1 launches (compacted queue)"}


def kernel_sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_per_launch(workload: str, kind: str):
    """HBM bytes per launch of one kernel kind on one workload from the
    committed counter profile (FETCH_SIZE + WRITE_SIZE, each scaled by the copy
    probe), or None when the profile is missing or was taken on other kernel
    sources."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None
    digest = kernel_sources_digest()
    for line in open(path):
        if not line.startswith("traffic:"):
            continue
        vals = dict(kv.split("=", 1) for kv in line[len("traffic:"):].split())
        if vals.get("sources") == digest and vals.get("workload") == workload and vals.get("kernel") == kind:
            return float(vals["bytes_per_launch"])
    return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, name, seconds_budget: float = 20.0):
    """Time the FP64 oracle on a strided lattice sample of the workload; its
    rate per ray-bounce extrapolates to the full map."""
    from oracle import native, sbr
    threads = native.default_threads()
    stride = max(1, w.num_rays // 2000)
    while True:
        p = sbr.TraceParams(num_rays=w.num_rays, max_depth=w.max_depth, ray_begin=0, ray_stride=stride)
        t0 = time.perf_counter()
        r = sbr.trace(w.scene, w.tx[0], p, grid=w.grid, record=True, threads=threads)
        dt = time.perf_counter() - t0
        segs = int(sum(int((h != -2).sum()) for h in r.hit_tri))
        if dt > seconds_budget / 3 or stride == 1:
            break
        stride = max(1, int(stride * dt / seconds_budget))
    rate = segs / dt
    return {"value": rate / 1e6, "unit": "M ray-bounces/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "%s coverage map, lattice rays 0, %d, 2*%d, ... of %d (%d rays, %d ray-bounces, depth %d), "
                      "%.1f s on %d threads; brute-force all-triangle intersection" % (
                          name, stride, stride, w.num_rays, len(r.ray_idx), segs, w.max_depth, dt, threads)}


def coverage_bench(rt, ctx, torch, w, name, steps, warmup):
    """Times `steps` coverage maps of workload w after `warmup`, with per-launch
    events; returns (result dict, scene)."""
    import ctypes

    import numpy as np
    from paper_2303_11103_amd._lib import check, lib
    dev = ctx.torch_device
    t0 = time.perf_counter()
    scene = rt.Scene.from_scenegen(ctx, w.scene)
    scene_s = time.perf_counter() - t0
    info = scene.info()
    p = rt.TraceParams(w.scene.freq_hz, w.max_depth, w.num_rays)
    tx = w.tx[0]
    nd = w.max_depth + 1
    out = {"gain": torch.empty((w.grid.ny, w.grid.nx), dtype=torch.float32, device=dev),
           "hits": torch.empty((w.grid.ny, w.grid.nx), dtype=torch.int32, device=dev),
           "gain_db": torch.empty((w.grid.ny, w.grid.nx), dtype=torch.float32, device=dev),
           "ray_bounces": torch.empty(nd, dtype=torch.int64, device=dev)}
    log("bench: %s, %d triangles, %d rays, depth %d, BVH %d nodes (build %.1f ms)" % (
        name, w.scene.nt, w.num_rays, w.max_depth, info["bvh_nodes"], info["build_ms"]))
    for _ in range(warmup):
        rt.coverage_map(ctx, scene, p, tx, w.grid, out=out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    check(lib.rt_profile_enable(ctx.h, 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for i in range(steps):
        rt.coverage_map(ctx, scene, p, tx, w.grid, out=out)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    check(lib.rt_profile_enable(ctx.h, 0))
    launches = (ctypes.c_int64 * nd)()
    kms = (ctypes.c_double * nd)()
    check(lib.rt_profile_read(ctx.h, nd, launches, kms))
    ms_step = (t1 - t0) * 1e3 / steps
    step_ms = [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]
    rb_depth = out["ray_bounces"].cpu().numpy().astype(np.int64)
    ray_bounces = int(rb_depth.sum())
    value = ray_bounces / (ms_step / 1e3) / 1e6
    log("bench: %s %.3f ms/step (median event %.3f), %d ray-bounces/step -> %.1f M ray-bounces/s" % (
        name, ms_step, statistics.median(step_ms), ray_bounces, value))

    # work counters: one extra, untimed map with per-ray counters
    work = torch.zeros(4 * nd, dtype=torch.int64, device=dev)
    g2 = torch.empty_like(out["gain"])
    h2 = torch.empty_like(out["hits"])
    pc, tc, rc, gc = p.c(), rt.rt.device_struct(tx), rt.rt.device_struct(w.rx_ant), rt.rt.grid_struct(w.grid)
    ctx._bind_stream()
    check(lib.rt_coverage_work(ctx.h, scene.h, ctypes.byref(pc), ctypes.byref(tc), ctypes.byref(rc),
                               ctypes.byref(gc), ctypes.c_void_p(g2.data_ptr()), ctypes.c_void_p(h2.data_ptr()),
                               ctypes.c_void_p(work.data_ptr())))
    wk = work.cpu().numpy().reshape(4, nd).astype(np.float64)
    # the kernels process every ray of a depth, except at the last depth the rays
    # dropped beforehand because they cannot deposit there
    assert np.array_equal(wk[0, :-1].astype(np.int64), rb_depth[:-1]) and wk[0, -1] <= rb_depth[-1], (wk[0], rb_depth)
    rays, nodes, boxes, tris = wk
    flops_depth = FLOP_BOX * boxes + FLOP_TRI * tris + FLOP_RAY_BOUNCE * rays
    launches = np.asarray(list(launches), dtype=np.float64) / steps   # per step, per depth
    kms = np.asarray(list(kms)) / steps                               # ms per step, per depth
    kinds = {"first": [0], "bounce": list(range(1, nd))}
    per_kind = {}
    for kind, ds in kinds.items():
        if not ds:
            continue
        ms = float(kms[ds].sum())
        nl = float(launches[ds].sum())
        fl = float(flops_depth[ds].sum())
        per_kind[kind] = {"ms_per_step": round(ms, 4), "launches_per_step": int(round(nl)),
                          "avg_launch_ms": round(ms / nl, 5), "flop_per_step": fl,
                          "flop_per_launch": fl / nl,
                          "achieved_tflops": round(fl / (ms / 1e3) / 1e12, 3),
                          "frac": round(fl / (ms / 1e3) / 1e12 / PEAK_ALU_TFLOPS, 4)}
    dom = max(per_kind, key=lambda k: per_kind[k]["ms_per_step"])
    d = per_kind[dom]
    kernel_ms_total = float(kms.sum())
    achieved_all = float(flops_depth.sum()) / (kernel_ms_total / 1e3) / 1e12
    roofline = {
        "bound": "alu",
        "achieved": d["achieved_tflops"],
        "peak": PEAK_ALU_TFLOPS,
        "unit": "TFLOP/s",
        "frac": d["frac"],
        "traffic": traffic_per_launch(name, dom),
        "kernel": KERNEL_KIND[dom],
        "kernel_share_of_step": round(d["ms_per_step"] / kernel_ms_total, 3),
        "avg_launch_ms": d["avg_launch_ms"],
        "flop_per_launch": d["flop_per_launch"],
        "per_unit_flop": {"box_test": FLOP_BOX, "triangle_test": FLOP_TRI, "ray_bounce": FLOP_RAY_BOUNCE},
        "kernels": per_kind,
        "all_launches": {"kernel_ms_per_step": round(kernel_ms_total, 4), "achieved": round(achieved_all, 3),
                         "frac": round(achieved_all / PEAK_ALU_TFLOPS, 4),
                         "kernel_ms_per_depth": [round(float(x), 4) for x in kms]},
        "node_visits_per_ray_bounce": round(float(nodes.sum() / rays.sum()), 3),
        "box_tests_per_ray_bounce": round(float(boxes.sum() / rays.sum()), 3),
        "tri_tests_per_ray_bounce": round(float(tris.sum() / rays.sum()), 3),
        "flop_per_ray_bounce": round(float(flops_depth.sum() / rays.sum()), 1),
        "rays_per_depth": [int(x) for x in rays],
        "rays_dropped_before_last_depth": int(rb_depth[-1] - rays[-1]),
        "node_visits_per_depth": [int(x) for x in nodes],
        "box_tests_per_depth": [int(x) for x in boxes],
        "tri_tests_per_depth": [int(x) for x in tris],
    }
    log("bench: %s dominant kernel %s: %.4f ms/launch, %.2f TFLOP/s (%.1f%% of %.1f); all launches %.3f ms/step, "
        "%.2f TFLOP/s" % (name, dom, d["avg_launch_ms"], d["achieved_tflops"], 100 * d["frac"], PEAK_ALU_TFLOPS,
                          kernel_ms_total, achieved_all))
    res = {"value": value, "ms_per_step": ms_step, "coverage_map_ms_median": statistics.median(step_ms),
           "coverage_map_ms_events": [round(x, 4) for x in step_ms],
           "ray_bounces_per_step": ray_bounces, "roofline": roofline,
           "bvh_nodes": info["bvh_nodes"], "bvh_build_ms": round(info["build_ms"], 1),
           "scene_create_s": round(scene_s, 2)}
    return res, scene


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-urban", action="store_true", help="skip the urban-canyon secondary measurement")
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

    import torch

    import paper_2303_11103_amd as rt
    import scenegen as sg

    ctx = rt.Context(0)
    c = sg.city_workload()
    city, city_scene = coverage_bench(rt, ctx, torch, c, "city", args.steps, args.warmup)
    city_scene.close()
    if args.copy_probe:
        # a plain device copy of known size: the HBM counters of the profile runs
        # are scaled by what they read for it
        src = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device=ctx.torch_device)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    result = {
        "metric": BJ_METRIC,
        "value": round(city["value"], 2),
        "unit": "M ray-bounces/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(city["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 geometry + f32 field",
        "data": "synthetic",
        "config": {"workload": "large procedural city coverage map: 50x50 blocks of extruded convex polygons "
                               "(%d tris, 3 materials), TR 38.901 tx, 1e8 rays, depth 5, 2000x2000 cells of 1 m, "
                               "28 GHz" % c.scene.nt,
                   "num_rays": c.num_rays, "max_depth": c.max_depth, "grid": [c.grid.ny, c.grid.nx],
                   "triangles": int(c.scene.nt)},
        "coverage_map_ms": round(city["coverage_map_ms_median"], 4),
        "coverage_map_ms_events": city["coverage_map_ms_events"],
        "ray_bounces_per_step": city["ray_bounces_per_step"],
        "bvh": {"nodes": city["bvh_nodes"], "build_ms": city["bvh_build_ms"],
                "scene_create_s": city["scene_create_s"]},
        "roofline": city["roofline"],
    }

    w = sg.urban_workload()
    if not args.no_urban:
        urban, scene = coverage_bench(rt, ctx, torch, w, "urban", 2 * args.steps, args.warmup)
        result["urban"] = {"workload": "urban canyon coverage map: 8x8 boxes (770 tris), 1e7 rays, depth 3, "
                                       "400x400 cells of 1 m, 3.5 GHz",
                           "M_ray_bounces_per_s": round(urban["value"], 2),
                           "coverage_map_ms": round(urban["coverage_map_ms_median"], 4),
                           "ms_per_step": round(urban["ms_per_step"], 4),
                           "ray_bounces_per_step": urban["ray_bounces_per_step"],
                           "roofline": urban["roofline"]}
    else:
        scene = rt.Scene.from_scenegen(ctx, w.scene)

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
        log("bench: timing the FP64 oracle on a lattice sample of the city ...")
        cb = cpu_baseline(c, "large city")
        cb["full_map_s_extrapolated"] = round(city["ray_bounces_per_step"] / (cb["value"] * 1e6), 1)
        cb["vs_gpu"] = round(city["value"] / cb["value"], 1)
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
    # first-order diffraction: the 256 receivers of the differentiation case
    # (512 wedges), then 1024 street receivers of the large city
    rt.compute_diffraction(ctx, sd, d.scene.freq_hz, d.tx, d.rx, P=64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    od = rt.compute_diffraction(ctx, sd, d.scene.freq_hz, d.tx, d.rx, P=64)
    torch.cuda.synchronize()
    res["diffraction"] = {"workload": "first-order diffraction, urban differentiation case, 256 rx x %d wedges" %
                                      sd.info()["num_wedges"],
                          "ms": round((time.perf_counter() - t0) * 1e3, 3), "paths": int(od["num_paths"].sum())}
    log("bench: diffraction %s" % res["diffraction"])
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
    # scattered paths: 16 receivers of the differentiation case, 1e6 rays, depth 3
    ps = rt.TraceParams(d.scene.freq_hz, d.max_depth, d.num_rays)
    rt.compute_scattering(ctx, ss, ps, d.tx, d.rx[:16], P=400_000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    osp = rt.compute_scattering(ctx, ss, ps, d.tx, d.rx[:16], P=400_000)
    torch.cuda.synchronize()
    res["scattering"]["paths_workload"] = "scattered paths, differentiation case, 1e6 rays, depth 3, 16 rx"
    res["scattering"]["paths_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    res["scattering"]["scattered_paths"] = int(osp["num_paths"].sum())
    log("bench: scattered paths %.2f ms, %d paths" % (res["scattering"]["paths_ms"],
                                                      res["scattering"]["scattered_paths"]))
    del osp
    ss.close()
    # large procedural city: paths to the 4096 street receivers
    c = sg.city_workload()
    sc = rt.Scene.from_scenegen(ctx, c.scene)
    res["city"] = {"workload": "large city paths: %d street receivers, 1e8 rays, depth 5, reception spheres "
                               "(kappa 2)" % len(c.rx)}
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
    crx = c.rx[:1024]
    rt.compute_diffraction(ctx, sc, c.scene.freq_hz, c.tx, crx[:8], P=256)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    odc = rt.compute_diffraction(ctx, sc, c.scene.freq_hz, c.tx, crx, P=256)
    torch.cuda.synchronize()
    res["city"]["diffraction_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    res["city"]["diffraction_rx"] = len(crx)
    res["city"]["wedges"] = sc.info()["num_wedges"]
    res["city"]["diffraction_paths"] = int(odc["num_paths"].sum())
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
    # the fallback call on the test transmitters: surrogate maps whose marked cells
    # are answered by the ray tracer (timed as one call per batch of test maps)
    from types import SimpleNamespace
    test_devs = [SimpleNamespace(pos=tuple(float(x) for x in t), yaw=0.0, pitch=0.0, roll=0.0, pattern=0)
                 for t in tx_np[te]]
    fb_out = torch.empty((len(test_devs), grid.ny, grid.nx), dtype=torch.float32, device=dev)
    m.predict_maps_fallback(scene, p, test_devs[:4], grid, fb, out=fb_out[:4])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fb_out, n_fb = m.predict_maps_fallback(scene, p, test_devs, grid, fb, out=fb_out)
    torch.cuda.synchronize()
    fb_s = time.perf_counter() - t0
    fb_maps_s = len(test_devs) / fb_s
    test_rmse_fb = S.rmse_db(fb_out, maps[te], mask[te])
    res = {
        "maps_per_s": round(sur_maps_s, 1),
        "ray_tracer_maps_per_s": round(rt_maps_s, 1),
        "speedup": round(sur_maps_s / rt_maps_s, 1),
        "test_rmse_db": round(test_rmse, 3),
        "test_rmse_db_outside_fallback": round(test_rmse_nofb, 3),
        "val_rmse_db": round(val_rmse, 3),
        "fallback_cell_fraction": round(fb_frac, 4),
        "fallback_cells": n_fb,
        # measured: rt_mlp_predict_maps_fallback over the test transmitters
        "maps_per_s_with_fallback": round(fb_maps_s, 1),
        "speedup_with_fallback": round(fb_maps_s / rt_maps_s, 2),
        "test_rmse_db_with_fallback": round(test_rmse_fb, 3),
        "train_steps": rep.steps, "train_s": round(rep.seconds, 1), "train_final_loss": round(rep.final_loss, 3),
        "dataset": "%d tx (%d train / %d val / %d test), 200x200 cells of 2 m, 1e7 rays, depth 3" % (
            n_tx, n_tr, n_val, n_test),
    }
    log("bench: surrogate %s" % res)
    m.close()
    return res


if __name__ == "__main__":
    main()
