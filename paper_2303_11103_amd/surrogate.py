"""Learned coverage-map surrogate: dataset generation with the ray tracer,
training and inference with the library's bf16 MFMA kernels (C ABI
``rt_mlp_*``), and the fallback mask that hands poorly predicted cells back to
the ray tracer.  Python only sequences calls; every computation runs in the
HIP library.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import torch

from . import _lib as L
from ._lib import check, lib
from .rt import Context, Scene, TraceParams, coverage_map, grid_struct


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def param_count() -> int:
    n = ctypes.c_int64()
    check(lib.rt_mlp_param_count(ctypes.byref(n)))
    return int(n.value)


class MLP:
    """Handle on the library's Fourier-feature MLP (weights live on the GPU)."""

    def __init__(self, ctx: Context, batch=32768, ff_scale=4.0, seed=0, center=(0, 0, 0, 0, 0),
                 half=(1, 1, 1, 1, 1), ff_scale_cell=0.0, prior=None, ff_rows_tx=0, ff_rows_rel=0, ff_scale_rel=0.0):
        """ff_scale: Fourier std on the transmitter inputs; ff_scale_cell on the
        cell inputs (0 = ff_scale); ff_rows_tx / ff_rows_rel > 0 give a
        structured matrix with transmitter-only and relative-position rows
        (std ff_scale_rel); prior = (freq_hz, rx_z) adds the free-space gain of
        the link to the output (the network learns the residual)."""
        self.ctx = ctx
        cfg = L.rt_mlp_config()
        cfg.batch = int(batch)
        cfg.ff_scale = float(ff_scale)
        cfg.ff_scale_cell = float(ff_scale_cell)
        cfg.ff_rows_tx = int(ff_rows_tx)
        cfg.ff_rows_rel = int(ff_rows_rel)
        cfg.ff_scale_rel = float(ff_scale_rel)
        if prior is not None:
            cfg.prior_freq_hz = float(prior[0])
            cfg.prior_rx_z = float(prior[1])
        cfg.seed = int(seed)
        for i in range(5):
            cfg.in_center[i] = float(center[i])
            cfg.in_half[i] = float(half[i])
        self.batch = int(batch)
        h = ctypes.c_void_p()
        ctx._bind_stream()
        check(lib.rt_mlp_create(ctx.h, ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h
        self.P = param_count()
        dev = ctx.torch_device
        self._loss = torch.zeros(1, dtype=torch.float32, device=dev)

    def get_params(self):
        p = torch.empty(self.P, dtype=torch.float32, device=self.ctx.torch_device)
        ff = torch.empty((64, 5), dtype=torch.float32, device=self.ctx.torch_device)
        self.ctx._bind_stream()
        check(lib.rt_mlp_get_params(self.h, _p(p), _p(ff)))
        return p, ff

    def set_params(self, p, ff):
        p = p.contiguous().float()
        ff = ff.contiguous().float()
        self.ctx._bind_stream()
        check(lib.rt_mlp_set_params(self.h, _p(p), _p(ff)))

    def forward(self, v):
        v = v.contiguous().float()
        y = torch.empty(v.shape[0], dtype=torch.float32, device=v.device)
        self.ctx._bind_stream()
        check(lib.rt_mlp_forward(self.h, _p(v), v.shape[0], _p(y)))
        return y

    def grad(self, v, t, m):
        g = torch.empty(self.P, dtype=torch.float32, device=v.device)
        loss = torch.empty(1, dtype=torch.float32, device=v.device)
        self.ctx._bind_stream()
        check(lib.rt_mlp_grad(self.h, _p(v.contiguous()), _p(t.contiguous()), _p(m.contiguous()), v.shape[0], _p(g),
                              _p(loss)))
        return g, loss

    def train_step(self, v, t, m, lr):
        self.ctx._bind_stream()
        check(lib.rt_mlp_train_step(self.h, _p(v), _p(t), _p(m), v.shape[0], float(lr), _p(self._loss)))
        return self._loss

    def valid_index(self, mask):
        """Flat positions of the nonzero entries of a uint8 mask (ascending), as an
        int32 tensor holding the uint32 values."""
        mask = mask.contiguous()
        n = mask.numel()
        count = ctypes.c_int64()
        self.ctx._bind_stream()
        # count first (capacity 0 reports RT_ERR_CAPACITY with the count), then write
        st = lib.rt_mlp_valid_index(self.h, _p(mask), n, None, 0, ctypes.byref(count))
        if st not in (0, L.RT_ERR_CAPACITY):
            check(st)
        idx = torch.empty(max(1, count.value), dtype=torch.int32, device=mask.device)
        check(lib.rt_mlp_valid_index(self.h, _p(mask), n, _p(idx), count.value, ctypes.byref(count)))
        return idx[:count.value]

    def sample_batch(self, maps, index, tx, grid, seed, step, n, out=None):
        dev = maps.device
        if out is None:
            out = (torch.empty((n, 5), dtype=torch.float32, device=dev), torch.empty(n, dtype=torch.float32, device=dev),
                   torch.empty(n, dtype=torch.float32, device=dev))
        v, t, m = out
        g = grid_struct(grid)
        self.ctx._bind_stream()
        check(lib.rt_mlp_sample_batch(self.h, _p(maps), _p(index), index.numel(), _p(tx), tx.shape[0],
                                      ctypes.byref(g), int(seed), int(step), _p(v), _p(t), _p(m), n))
        return v, t, m

    def predict_maps(self, tx, grid, out=None):
        tx = tx.contiguous().float()
        if out is None:
            out = torch.empty((tx.shape[0], grid.ny, grid.nx), dtype=torch.float32, device=tx.device)
        g = grid_struct(grid)
        self.ctx._bind_stream()
        check(lib.rt_mlp_predict_maps(self.h, _p(tx), tx.shape[0], ctypes.byref(g), _p(out)))
        return out

    def predict_maps_fallback(self, scene: Scene, params: TraceParams, txs, grid, fallback, rx_ant=None,
                              out=None):
        """Maps [T][ny][nx] (dB) for the transmitters txs (objects with pos, yaw,
        pitch, roll, pattern): the surrogate's prediction, with the cells where
        the uint8 tensor fallback [ny][nx] is nonzero answered by the ray tracer.
        Returns (maps, number of fallback cells)."""
        from types import SimpleNamespace

        from .rt import device_struct
        T = len(txs)
        dev = self.ctx.torch_device
        if out is None:
            out = torch.empty((T, grid.ny, grid.nx), dtype=torch.float32, device=dev)
        rx_ant = rx_ant or SimpleNamespace(pos=(0.0, 0.0, 0.0), yaw=0.0, pitch=0.0, roll=0.0, pattern=0)
        fb = fallback.to(torch.uint8).contiguous()
        tx_arr = (L.rt_device * T)(*[device_struct(t) for t in txs])
        p, r, g = params.c(), device_struct(rx_ant), grid_struct(grid)
        n = ctypes.c_int64()
        self.ctx._bind_stream()
        check(lib.rt_mlp_predict_maps_fallback(self.h, scene.h, ctypes.byref(p), tx_arr, T, ctypes.byref(r),
                                               ctypes.byref(g), _p(fb), _p(out), ctypes.byref(n)))
        return out, int(n.value)

    def close(self):
        if self.h:
            lib.rt_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ray_traced_maps(ctx: Context, scene: Scene, params: TraceParams, tx_pos, grid, min_hits=16):
    """Coverage maps (dB) of every transmitter position (float32 [T][3]) by the
    ray tracer, and the mask of cells with at least ``min_hits`` crossings."""
    from types import SimpleNamespace
    T = len(tx_pos)
    dev = ctx.torch_device
    maps = torch.empty((T, grid.ny, grid.nx), dtype=torch.float32, device=dev)
    mask = torch.empty((T, grid.ny, grid.nx), dtype=torch.uint8, device=dev)
    buf = {"gain": torch.empty((grid.ny, grid.nx), dtype=torch.float32, device=dev),
           "hits": torch.empty((grid.ny, grid.nx), dtype=torch.int32, device=dev)}
    for k in range(T):
        tx = SimpleNamespace(pos=tuple(float(x) for x in tx_pos[k]), yaw=0.0, pitch=0.0, roll=0.0, pattern=0)
        buf["gain_db"] = maps[k]
        coverage_map(ctx, scene, params, tx, grid, out=buf, want_stats=False)
        mask[k] = buf["hits"] >= min_hits
    return maps, mask


@dataclass
class TrainReport:
    steps: int
    seconds: float
    final_loss: float


def train(mlp: MLP, maps, mask, tx, grid, steps=2000, lr=1e-3, seed=1, log_every=0):
    """Adam with a cosine learning-rate schedule on batches drawn uniformly from
    the usable cells (mask != 0) of the maps."""
    import time
    n = mlp.batch
    dev = maps.device
    index = mlp.valid_index(mask)
    bufs = (torch.empty((n, 5), dtype=torch.float32, device=dev), torch.empty(n, dtype=torch.float32, device=dev),
            torch.empty(n, dtype=torch.float32, device=dev))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = None
    for s in range(steps):
        v, t, m = mlp.sample_batch(maps, index, tx, grid, seed, s, n, out=bufs)
        cur = lr * 0.5 * (1.0 + math.cos(math.pi * s / steps))
        loss = mlp.train_step(v, t, m, max(cur, lr * 1e-3))
        if log_every and (s % log_every == 0 or s == steps - 1):
            print("train step %d loss %.3f" % (s, float(loss)), flush=True)
    torch.cuda.synchronize()
    return TrainReport(steps, time.perf_counter() - t0, float(loss) if loss is not None else float("nan"))


def rmse_db(pred, maps, mask):
    """Root mean squared error in dB over masked-in cells."""
    sel = mask.bool()
    d = (pred - maps)[sel]
    return float(torch.sqrt(torch.mean(d * d)))


def fallback_mask(pred, maps, mask, threshold_db=6.0):
    """Cells whose validation error averaged over transmitters exceeds the
    threshold (these are answered by the ray tracer)."""
    sel = mask.float()
    err = ((pred - maps) ** 2 * sel).sum(0) / sel.sum(0).clamp_min(1.0)
    return torch.sqrt(err) > threshold_db
