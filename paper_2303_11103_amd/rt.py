"""Python facade over the C ABI: device tensors come from PyTorch, every step
of the computation runs in the HIP library.

Device buffers are torch tensors on the context's GPU; work is enqueued on
torch's current stream for that device.
"""
from __future__ import annotations

import contextlib
import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L
from ._lib import check, lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


@dataclass
class TraceParams:
    freq_hz: float
    max_depth: int
    num_rays: int
    t_min: float = 1e-4
    ray_begin: int = 0
    ray_stride: int = 1
    max_paths_per_rx: int = 64
    cand_mode: int = 0         # 0 = every candidate for every receiver, 1 = reception spheres
    sphere_kappa: float = 2.0

    def c(self):
        return L.rt_trace_params(float(self.freq_hz), int(self.max_depth), int(self.max_paths_per_rx),
                                 int(self.num_rays), float(self.t_min), int(self.ray_begin), int(self.ray_stride),
                                 int(self.cand_mode), float(self.sphere_kappa))

    def traced(self) -> int:
        return (self.num_rays - self.ray_begin + self.ray_stride - 1) // self.ray_stride


def device_struct(dev) -> L.rt_device:
    """rt_device from any object with pos, yaw, pitch, roll, pattern (pol defaults to V)."""
    d = L.rt_device()
    for i in range(3):
        d.pos[i] = float(dev.pos[i])
    d.yaw, d.pitch, d.roll = float(dev.yaw), float(dev.pitch), float(dev.roll)
    d.pattern = int(getattr(dev, "pattern", 0))
    d.pol = int(getattr(dev, "pol", 0))
    return d


def grid_struct(g) -> L.rt_grid:
    return L.rt_grid(float(g.x0), float(g.y0), float(g.cell), float(g.z), int(g.nx), int(g.ny))


class Context:
    def __init__(self, device: int = 0):
        self.device = int(device)
        self.torch_device = torch.device("cuda", self.device)
        h = ctypes.c_void_p()
        check(lib.rt_create(ctypes.byref(h), self.device))
        self.h = h

    def _bind_stream(self):
        s = torch.cuda.current_stream(self.torch_device).cuda_stream
        check(lib.rt_set_stream(self.h, ctypes.c_void_p(s)))

    def synchronize(self):
        check(lib.rt_synchronize(self.h))

    def close(self):
        if self.h:
            lib.rt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Scene:
    """A triangle mesh with materials on the device (BVH built at creation)."""

    def __init__(self, ctx: Context, V, F, tri_mat, materials):
        self.ctx = ctx
        V = np.ascontiguousarray(V, dtype=np.float32)
        F = np.ascontiguousarray(F, dtype=np.int32)
        tri_mat = np.ascontiguousarray(tri_mat, dtype=np.int32)
        mats = np.ascontiguousarray(materials, dtype=np.float32).reshape(-1, 2)
        marr = (L.rt_material * len(mats))(*[L.rt_material(float(e), float(s)) for e, s in mats])
        h = ctypes.c_void_p()
        check(lib.rt_scene_create(ctx.h, V.ctypes.data_as(ctypes.c_void_p), V.shape[0],
                                  F.ctypes.data_as(ctypes.c_void_p), F.shape[0],
                                  tri_mat.ctypes.data_as(ctypes.c_void_p), marr, len(mats), ctypes.byref(h)))
        self.h = h
        self.nt = int(F.shape[0])
        self.nm = len(mats)
        self.materials = mats.copy()   # the table the library holds (float32 [nm][2])

    @classmethod
    def from_scenegen(cls, ctx, s):
        return cls(ctx, s.V, s.F, s.tri_mat, s.materials)

    def set_scattering(self, S, seed=0):
        """Lambertian scattering coefficient per material (see rt_scene_set_scattering)."""
        s = np.ascontiguousarray(np.asarray(S, dtype=np.float32).reshape(-1))
        check(lib.rt_scene_set_scattering(self.h, s.ctypes.data_as(ctypes.c_void_p), int(s.size),
                                          ctypes.c_uint64(int(seed))))

    def set_materials(self, materials):
        mats = np.ascontiguousarray(materials, dtype=np.float32).reshape(-1, 2)
        marr = (L.rt_material * len(mats))(*[L.rt_material(float(e), float(s)) for e, s in mats])
        check(lib.rt_scene_set_materials(self.h, marr, len(mats)))
        self.materials = mats.copy()

    @contextlib.contextmanager
    def materials_set_to(self, materials):
        """Within the block the scene holds ``materials``; the previous table
        is restored on exit.  Launches take the table by value, so kernels
        enqueued inside the block keep it."""
        prev = self.materials.copy()
        self.set_materials(materials)
        try:
            yield self
        finally:
            self.set_materials(prev)

    def info(self) -> dict:
        inf = L.rt_scene_info_t()
        check(lib.rt_scene_info(self.h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in L.rt_scene_info_t._fields_}

    def wedges(self) -> np.ndarray:
        """Diffraction wedges, float64 [count, 16]: a[3], e[3], t0[3], n0[3],
        length, n, 0-face id, n-face id."""
        n = ctypes.c_int32()
        check(lib.rt_scene_wedges(self.h, 0, None, ctypes.byref(n)))
        out = np.empty((max(n.value, 1), 16), dtype=np.float64)
        check(lib.rt_scene_wedges(self.h, n.value, out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)))
        return out[:n.value]

    def face_ids(self) -> np.ndarray:
        out = np.empty(self.nt, dtype=np.int32)
        check(lib.rt_scene_face_ids(self.h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def close(self):
        if self.h:
            lib.rt_scene_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fibonacci_directions(ctx: Context, num_rays, begin=0, stride=1, count=None):
    if count is None:
        count = (num_rays - begin + stride - 1) // stride
    out = torch.empty((count, 3), dtype=torch.float64, device=ctx.torch_device)
    ctx._bind_stream()
    check(lib.rt_fibonacci_directions(ctx.h, num_rays, begin, stride, count, _ptr(out)))
    return out


def trace_record(ctx: Context, scene: Scene, params: TraceParams, tx):
    n = params.traced()
    tri = torch.empty((params.max_depth + 1, n), dtype=torch.int32, device=ctx.torch_device)
    t = torch.empty((params.max_depth + 1, n), dtype=torch.float64, device=ctx.torch_device)
    ctx._bind_stream()
    p, d = params.c(), device_struct(tx)
    check(lib.rt_trace_record(ctx.h, scene.h, ctypes.byref(p), ctypes.byref(d), _ptr(tri), _ptr(t)))
    return tri, t


def coverage_map(ctx: Context, scene: Scene, params: TraceParams, tx, grid, rx_ant=None, out=None, want_db=True,
                 want_stats=True):
    """Returns dict(gain, hits, gain_db, ray_bounces) of device tensors."""
    if out is None:
        out = {"gain": torch.empty((grid.ny, grid.nx), dtype=torch.float32, device=ctx.torch_device),
               "hits": torch.empty((grid.ny, grid.nx), dtype=torch.int32, device=ctx.torch_device)}
        if want_db:
            out["gain_db"] = torch.empty((grid.ny, grid.nx), dtype=torch.float32, device=ctx.torch_device)
        if want_stats:
            out["ray_bounces"] = torch.empty(params.max_depth + 1, dtype=torch.int64, device=ctx.torch_device)
    from types import SimpleNamespace
    rx_ant = rx_ant or SimpleNamespace(pos=(0.0, 0.0, 0.0), yaw=0.0, pitch=0.0, roll=0.0, pattern=0)
    ctx._bind_stream()
    p, t, r, g = params.c(), device_struct(tx), device_struct(rx_ant), grid_struct(grid)
    check(lib.rt_coverage_map(ctx.h, scene.h, ctypes.byref(p), ctypes.byref(t), ctypes.byref(r), ctypes.byref(g),
                              _ptr(out["gain"]), _ptr(out["hits"]), _ptr(out.get("gain_db")),
                              _ptr(out.get("ray_bounces"))))
    return out


def coverage_maps(ctx: Context, scene: Scene, params: TraceParams, txs, grid, rx_ant=None, want_db=False):
    """Coverage maps of several transmitters in one call: dict(gain, hits,
    gain_db) of device tensors [ntx, ny, nx]."""
    from types import SimpleNamespace
    n = len(txs)
    dev = ctx.torch_device
    out = {"gain": torch.empty((n, grid.ny, grid.nx), dtype=torch.float32, device=dev),
           "hits": torch.empty((n, grid.ny, grid.nx), dtype=torch.int32, device=dev)}
    if want_db:
        out["gain_db"] = torch.empty((n, grid.ny, grid.nx), dtype=torch.float32, device=dev)
    rx_ant = rx_ant or SimpleNamespace(pos=(0.0, 0.0, 0.0), yaw=0.0, pitch=0.0, roll=0.0, pattern=0)
    tx_arr = (L.rt_device * max(n, 1))(*[device_struct(t) for t in txs])
    ctx._bind_stream()
    p, r, g = params.c(), device_struct(rx_ant), grid_struct(grid)
    check(lib.rt_coverage_maps(ctx.h, scene.h, ctypes.byref(p), tx_arr, n, ctypes.byref(r), ctypes.byref(g),
                               _ptr(out["gain"]), _ptr(out["hits"]), _ptr(out.get("gain_db"))))
    return out


def compute_paths(ctx: Context, scene: Scene, params: TraceParams, txs, rxs):
    """Paths for every (tx, rx); returns dict of device tensors shaped [ntx, nrx, P, ...]."""
    ntx, nrx, P = len(txs), len(rxs), params.max_paths_per_rx
    fd = max(params.max_depth, 1)
    dev = ctx.torch_device
    o = {
        "a": torch.empty((ntx, nrx, P, 2), dtype=torch.float32, device=dev),
        "T": torch.empty((ntx, nrx, P, 2, 2, 2), dtype=torch.float32, device=dev),
        "tau": torch.empty((ntx, nrx, P), dtype=torch.float32, device=dev),
        "aod": torch.empty((ntx, nrx, P, 2), dtype=torch.float32, device=dev),
        "aoa": torch.empty((ntx, nrx, P, 2), dtype=torch.float32, device=dev),
        "depth": torch.empty((ntx, nrx, P), dtype=torch.int32, device=dev),
        "faces": torch.empty((ntx, nrx, P, fd), dtype=torch.int32, device=dev),
        "num_paths": torch.empty((ntx, nrx), dtype=torch.int32, device=dev),
    }
    tx_arr = (L.rt_device * ntx)(*[device_struct(t) for t in txs])
    rx_arr = (L.rt_device * nrx)(*[device_struct(r) for r in rxs])
    ctx._bind_stream()
    p = params.c()
    check(lib.rt_compute_paths(ctx.h, scene.h, ctypes.byref(p), tx_arr, ntx, rx_arr, nrx, _ptr(o["a"]), _ptr(o["T"]),
                               _ptr(o["tau"]), _ptr(o["aod"]), _ptr(o["aoa"]), _ptr(o["depth"]), _ptr(o["faces"]),
                               _ptr(o["num_paths"])))
    return o


def paths_power(ctx: Context, paths):
    """Received power per (tx, rx): float64 tensor [ntx, nrx] = sum |a|^2 over valid paths."""
    a, depth = paths["a"], paths["depth"]
    ntx, nrx, P = depth.shape
    out = torch.empty((ntx, nrx), dtype=torch.float64, device=a.device)
    ctx._bind_stream()
    check(lib.rt_paths_power(ctx.h, _ptr(a), _ptr(depth), ntx * nrx, P, _ptr(out)))
    return out


def compute_diffraction(ctx: Context, scene: Scene, freq_hz: float, txs, rxs, P: int = 64):
    """First-order diffraction paths for every (tx, rx); dict of device tensors
    shaped [ntx, nrx, P, ...] (a, T, tau, aod, aoa, wedge) and num_paths."""
    ntx, nrx = len(txs), len(rxs)
    dev = ctx.torch_device
    o = {
        "a": torch.empty((ntx, nrx, P, 2), dtype=torch.float32, device=dev),
        "T": torch.empty((ntx, nrx, P, 2, 2, 2), dtype=torch.float32, device=dev),
        "tau": torch.empty((ntx, nrx, P), dtype=torch.float32, device=dev),
        "aod": torch.empty((ntx, nrx, P, 2), dtype=torch.float32, device=dev),
        "aoa": torch.empty((ntx, nrx, P, 2), dtype=torch.float32, device=dev),
        "wedge": torch.empty((ntx, nrx, P), dtype=torch.int32, device=dev),
        "num_paths": torch.empty((ntx, nrx), dtype=torch.int32, device=dev),
    }
    tx_arr = (L.rt_device * ntx)(*[device_struct(t) for t in txs])
    rx_arr = (L.rt_device * nrx)(*[device_struct(r) for r in rxs])
    ctx._bind_stream()
    check(lib.rt_compute_diffraction(ctx.h, scene.h, float(freq_hz), tx_arr, ntx, rx_arr, nrx, int(P), _ptr(o["a"]),
                                     _ptr(o["T"]), _ptr(o["tau"]), _ptr(o["aod"]), _ptr(o["aoa"]), _ptr(o["wedge"]),
                                     _ptr(o["num_paths"])))
    return o


def compute_scattering(ctx: Context, scene: Scene, params: TraceParams, txs, rxs, P: int = 4096):
    """Diffusely scattered paths for every (tx, rx) (the scene's scattering
    coefficients, see Scene.set_scattering); dict of device tensors shaped
    [ntx, nrx, P, ...] (a, T, tau, aod, aoa, depth, ray, faces) and num_paths
    (int64).  Raises RTError (RT_ERR_CAPACITY) when a receiver has more than P."""
    ntx, nrx = len(txs), len(rxs)
    fd = max(params.max_depth, 1)
    dev = ctx.torch_device
    o = {
        "a": torch.empty((ntx, nrx, P, 2), dtype=torch.float32, device=dev),
        "T": torch.empty((ntx, nrx, P, 2, 2, 2), dtype=torch.float32, device=dev),
        "tau": torch.empty((ntx, nrx, P), dtype=torch.float32, device=dev),
        "aod": torch.empty((ntx, nrx, P, 2), dtype=torch.float32, device=dev),
        "aoa": torch.empty((ntx, nrx, P, 2), dtype=torch.float32, device=dev),
        "depth": torch.empty((ntx, nrx, P), dtype=torch.int32, device=dev),
        "ray": torch.empty((ntx, nrx, P), dtype=torch.int64, device=dev),
        "faces": torch.empty((ntx, nrx, P, fd), dtype=torch.int32, device=dev),
        "num_paths": torch.empty((ntx, nrx), dtype=torch.int64, device=dev),
    }
    tx_arr = (L.rt_device * ntx)(*[device_struct(t) for t in txs])
    rx_arr = (L.rt_device * nrx)(*[device_struct(r) for r in rxs])
    ctx._bind_stream()
    p = params.c()
    check(lib.rt_compute_scattering(ctx.h, scene.h, ctypes.byref(p), tx_arr, ntx, rx_arr, nrx, int(P), _ptr(o["a"]),
                                    _ptr(o["T"]), _ptr(o["tau"]), _ptr(o["aod"]), _ptr(o["aoa"]), _ptr(o["depth"]),
                                    _ptr(o["ray"]), _ptr(o["faces"]), _ptr(o["num_paths"])))
    return o


def coverage_diffraction(ctx: Context, scene: Scene, freq_hz: float, tx, grid, gain=None, rx_ant=None):
    """Adds the diffracted path gain at every cell centre to gain (a float32
    [ny, nx] device tensor, zeros when None) and returns it."""
    from types import SimpleNamespace
    if gain is None:
        gain = torch.zeros((grid.ny, grid.nx), dtype=torch.float32, device=ctx.torch_device)
    rx_ant = rx_ant or SimpleNamespace(pos=(0.0, 0.0, 0.0), yaw=0.0, pitch=0.0, roll=0.0, pattern=0)
    t, r, g = device_struct(tx), device_struct(rx_ant), grid_struct(grid)
    ctx._bind_stream()
    check(lib.rt_coverage_diffraction(ctx.h, scene.h, float(freq_hz), ctypes.byref(t), ctypes.byref(r),
                                      ctypes.byref(g), _ptr(gain)))
    return gain


def last_candidate_count(ctx: Context) -> int:
    n = ctypes.c_int64()
    check(lib.rt_last_candidate_count(ctx.h, ctypes.byref(n)))
    return int(n.value)


def coverage_grad(ctx: Context, scene: Scene, params: TraceParams, tx, grid, hit_tri, hit_t, region=None,
                  rx_ant=None):
    """(G, dG/dtheta) with G the linear path gain summed over the region's cells
    and theta = (eps_r, sigma) per material, tx yaw, tx pitch; the rays are
    fixed by the records (hit_tri, hit_t) of trace_record with the same params
    and tx.  Returns a float64 device tensor [1 + 2 nm + 2]."""
    from types import SimpleNamespace
    rx_ant = rx_ant or SimpleNamespace(pos=(0.0, 0.0, 0.0), yaw=0.0, pitch=0.0, roll=0.0, pattern=0)
    n = params.traced()
    if tuple(hit_tri.shape) != (params.max_depth + 1, n) or tuple(hit_t.shape) != (params.max_depth + 1, n):
        raise ValueError("hit records must be [max_depth + 1][traced rays]")
    hit_tri = hit_tri.contiguous().to(torch.int32)
    hit_t = hit_t.contiguous().to(torch.float64)
    if region is not None:
        region = region.contiguous().to(torch.uint8)
        if tuple(region.shape) != (grid.ny, grid.nx):
            raise ValueError("region must be [ny][nx]")
    out = torch.empty(2 * scene.nm + 3, dtype=torch.float64, device=ctx.torch_device)
    ctx._bind_stream()
    p, t, r, g = params.c(), device_struct(tx), device_struct(rx_ant), grid_struct(grid)
    check(lib.rt_coverage_grad(ctx.h, scene.h, ctypes.byref(p), ctypes.byref(t), ctypes.byref(r), ctypes.byref(g),
                               _ptr(region), _ptr(hit_tri), _ptr(hit_t), _ptr(out)))
    return out


def _host_f64(x, rows):
    """None or a contiguous float64 ctypes array of shape [rows][3]."""
    if x is None:
        return None, 0
    arr = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, 3))
    if rows is not None and arr.shape[0] != rows:
        raise ValueError("expected %d rows of 3 values" % rows)
    return arr, arr.shape[0]


def _cfr_args(paths, freq_hz, num_subcarriers, spacing, tx_el, rx_el, v_tx, v_rx, num_time_steps, fs):
    a = paths["a"].contiguous()
    ntx, nrx, P = a.shape[0], a.shape[1], a.shape[2]
    te, nte = _host_f64(tx_el, None)
    re, nre = _host_f64(rx_el, None)
    vt, _ = _host_f64(v_tx, ntx)
    vr, _ = _host_f64(v_rx, nrx)
    keep = (a, paths["tau"].contiguous(), paths["aod"].contiguous(), paths["aoa"].contiguous(),
            paths["depth"].contiguous().to(torch.int32), te, re, vt, vr)
    hp = lambda x: None if x is None else x.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    args = [ntx, nrx, P, _ptr(keep[0]), _ptr(keep[1]), _ptr(keep[2]), _ptr(keep[3]), _ptr(keep[4]), float(freq_hz),
            int(num_subcarriers), float(spacing), max(nte, 1), hp(te), max(nre, 1), hp(re), hp(vt), hp(vr),
            int(num_time_steps), float(fs or 0.0)]
    shape = (ntx, nrx, int(num_time_steps), max(nre, 1), max(nte, 1), int(num_subcarriers))
    return args, shape, keep


def combine_paths(*path_sets):
    """One path list of several kinds for paths_cfr / paths_cfr_adjoint:
    the outputs of compute_paths, compute_diffraction and compute_scattering
    for the same transmitters and receivers, concatenated along the slot axis
    (a, tau, aod, aoa, depth; a diffracted path counts as depth 1)."""
    keys = ("a", "tau", "aod", "aoa")
    out = {k: torch.cat([ps[k] for ps in path_sets], dim=2).contiguous() for k in keys}
    depth = []
    for ps in path_sets:
        if "depth" in ps:
            depth.append(ps["depth"].to(torch.int32))
        else:
            depth.append(torch.where(ps["wedge"] >= 0, 1, -1).to(torch.int32))
    out["depth"] = torch.cat(depth, dim=2).contiguous()
    if out["depth"].shape[2] >= 2 ** 31:
        raise ValueError("more than 2^31 - 1 path slots per receiver")
    return out


def paths_cfr(ctx: Context, paths, freq_hz, num_subcarriers=128, spacing=30e3, tx_el=None, rx_el=None, v_tx=None,
              v_rx=None, num_time_steps=1, fs=None):
    """Channel frequency responses of the paths of compute_paths (or of
    combine_paths over specular, diffracted and scattered paths): complex64
    tensor [ntx, nrx, T, nr_el, nt_el, K] (synthetic arrays from element
    offsets tx_el / rx_el [n][3] in metres, Doppler from velocities v_tx
    [ntx][3] / v_rx [nrx][3] in m/s, T time steps at fs Hz)."""
    args, shape, keep = _cfr_args(paths, freq_hz, num_subcarriers, spacing, tx_el, rx_el, v_tx, v_rx,
                                  num_time_steps, fs)
    H = torch.empty(shape + (2,), dtype=torch.float32, device=ctx.torch_device)
    ctx._bind_stream()
    check(lib.rt_paths_cfr(ctx.h, *args, _ptr(H)))
    return torch.view_as_complex(H)


def paths_cfr_adjoint(ctx: Context, paths, G, freq_hz, num_subcarriers=128, spacing=30e3, tx_el=None, rx_el=None,
                      v_tx=None, v_rx=None, num_time_steps=1, fs=None):
    """Coefficient adjoint g [ntx, nrx, P, 2] (float64) of an upstream
    gradient G (complex, H's shape; dL = Re(conj(G) dH))."""
    args, shape, keep = _cfr_args(paths, freq_hz, num_subcarriers, spacing, tx_el, rx_el, v_tx, v_rx,
                                  num_time_steps, fs)
    if tuple(G.shape) != shape:
        raise ValueError("G must have the shape of the responses %s" % (shape,))
    Gf = torch.view_as_real(G.to(torch.complex64).contiguous()).contiguous()
    a = paths["a"]
    g = torch.empty((a.shape[0], a.shape[1], a.shape[2], 2), dtype=torch.float64, device=ctx.torch_device)
    ctx._bind_stream()
    check(lib.rt_paths_cfr_adjoint(ctx.h, *args, _ptr(Gf), _ptr(g)))
    return g


def paths_coef_grad(ctx: Context, scene: Scene, params: TraceParams, tx, rxs, depth, faces, coef_adj):
    """sum over paths of Re(g da/dtheta) for theta = (eps_r, sigma) per
    material, tx xyz, yaw, pitch (delays held fixed); coef_adj [nrx, P, 2]."""
    nrx = len(rxs)
    depth = depth.contiguous().to(torch.int32)
    faces = faces.contiguous().to(torch.int32)
    coef_adj = coef_adj.contiguous().to(torch.float64)
    P = depth.shape[-1]
    grad = torch.empty(2 * scene.nm + 5, dtype=torch.float64, device=ctx.torch_device)
    rx_arr = (L.rt_device * nrx)(*[device_struct(r) for r in rxs])
    ctx._bind_stream()
    p, t = params.c(), device_struct(tx)
    check(lib.rt_paths_coef_grad(ctx.h, scene.h, ctypes.byref(p), ctypes.byref(t), rx_arr, nrx, P, _ptr(depth),
                                 _ptr(faces), _ptr(coef_adj), _ptr(grad)))
    return grad


def paths_power_grad(ctx: Context, scene: Scene, params: TraceParams, tx, rxs, depth, faces, dL_dP):
    """sum_r dL_dP[r] dP_r/dtheta for theta = (eps_r, sigma) per material, tx xyz, yaw, pitch (float64 tensor)."""
    nrx = len(rxs)
    depth = depth.contiguous().to(torch.int32)
    faces = faces.contiguous().to(torch.int32)
    dL_dP = dL_dP.contiguous().to(torch.float64)
    P = depth.shape[-1]
    grad = torch.empty(2 * scene.nm + 5, dtype=torch.float64, device=ctx.torch_device)
    rx_arr = (L.rt_device * nrx)(*[device_struct(r) for r in rxs])
    ctx._bind_stream()
    p, t = params.c(), device_struct(tx)
    check(lib.rt_paths_power_grad(ctx.h, scene.h, ctypes.byref(p), ctypes.byref(t), rx_arr, nrx, P, _ptr(depth),
                                  _ptr(faces), _ptr(dL_dP), _ptr(grad)))
    return grad
