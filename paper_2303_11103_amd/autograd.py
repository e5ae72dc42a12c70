"""Differentiable received power: a torch.autograd.Function whose forward
runs the library's shoot-and-bounce + image-method kernels and whose
backward runs the hand-written gradient kernel (rt_paths_power_grad) on the
face sequences kept from the forward pass (geometry and fields are
recomputed, not stored).

Parameters theta (float64, 2*nm + 5): (eps_r, sigma) of every material, then
the transmitter's x, y, z, yaw, pitch.  The paper learns materials (Sec.
III-A) and transmitter orientation (Sec. III-B) from gradients of this kind.

Every Function sets the materials of its theta only for the duration of its
own launches: the forward leaves the scene's table as it found it, and the
backward sets the table its forward used, so several forwards before one
backward each differentiate at their own theta.
"""
from __future__ import annotations

from types import SimpleNamespace

import torch

from . import rt


class ReceivedPower(torch.autograd.Function):
    """P_r = sum_p |a_p|^2 for every receiver r of one transmitter."""

    @staticmethod
    def forward(fctx, theta, ctx, scene, params, tx, rxs):
        th = theta.detach().to("cpu", torch.float64).numpy()
        nm = scene.nm
        mats = th[:2 * nm].reshape(nm, 2).copy()
        dev = SimpleNamespace(pos=tuple(float(x) for x in th[2 * nm:2 * nm + 3]), yaw=float(th[2 * nm + 3]),
                              pitch=float(th[2 * nm + 4]), roll=float(tx.roll), pattern=int(tx.pattern),
                              pol=int(getattr(tx, "pol", 0)))
        with scene.materials_set_to(mats):
            paths = rt.compute_paths(ctx, scene, params, [dev], rxs)
            power = rt.paths_power(ctx, paths)[0]
        fctx.save_for_backward(paths["depth"][0].clone(), paths["faces"][0].clone())
        fctx.rt = (ctx, scene, params, dev, rxs, mats)
        return power

    @staticmethod
    def backward(fctx, grad_power):
        depth, faces = fctx.saved_tensors
        ctx, scene, params, dev, rxs, mats = fctx.rt
        with scene.materials_set_to(mats):
            g = rt.paths_power_grad(ctx, scene, params, dev, rxs, depth, faces,
                                    grad_power.contiguous().to(torch.float64))
        return g, None, None, None, None, None


def received_power(theta, ctx, scene, params, tx, rxs):
    """Differentiable P_r (float64 tensor [nrx]) as a function of theta."""
    return ReceivedPower.apply(theta, ctx, scene, params, tx, rxs)


class CoverageRegionGain(torch.autograd.Function):
    """G = linear path gain of the coverage map summed over a region of cells,
    as a function of theta = ((eps_r, sigma) per material, tx yaw, tx pitch)
    (float64, 2*nm + 2).  The forward records the rays' hits and replays them
    with field tangents (rt_coverage_grad); G and dG/dtheta come from the same
    replay, and the backward scales the saved gradient."""

    @staticmethod
    def forward(fctx, theta, ctx, scene, params, tx, grid, region, rx_ant):
        th = theta.detach().to("cpu", torch.float64).numpy()
        nm = scene.nm
        dev = SimpleNamespace(pos=tuple(float(x) for x in tx.pos), yaw=float(th[2 * nm]), pitch=float(th[2 * nm + 1]),
                              roll=float(tx.roll), pattern=int(tx.pattern),
                              pol=int(getattr(tx, "pol", 0)))
        with scene.materials_set_to(th[:2 * nm].reshape(nm, 2)):
            hit_tri, hit_t = rt.trace_record(ctx, scene, params, dev)
            out = rt.coverage_grad(ctx, scene, params, dev, grid, hit_tri, hit_t, region=region, rx_ant=rx_ant)
        fctx.save_for_backward(out[1:].clone())
        return out[0].clone()

    @staticmethod
    def backward(fctx, grad_g):
        (g,) = fctx.saved_tensors
        return grad_g.to(torch.float64) * g, None, None, None, None, None, None, None


def coverage_region_gain(theta, ctx, scene, params, tx, grid, region=None, rx_ant=None):
    """Differentiable summed path gain (float64 scalar tensor) of the region
    cells (uint8 mask [ny][nx], None: every cell) as a function of theta."""
    return CoverageRegionGain.apply(theta, ctx, scene, params, tx, grid, region, rx_ant)


class ChannelFrequencyResponse(torch.autograd.Function):
    """Channel frequency responses H (complex64 [nrx, T, nr_el, nt_el, K]) of
    one transmitter's paths as a function of the materials theta = (eps_r,
    sigma) per material (float64, 2*nm); Sec. III-A learns materials from such
    responses.  Backward: the adjoint of the response map gives every path's
    coefficient adjoint (rt_paths_cfr_adjoint), and the coefficient gradient
    kernel turns it into d/dtheta (rt_paths_coef_grad); the paths' geometry and
    delays do not depend on the materials."""

    @staticmethod
    def forward(fctx, theta, ctx, scene, params, tx, rxs, cfr_kw):
        nm = scene.nm
        mats = theta.detach().to("cpu", torch.float64).numpy().reshape(nm, 2).copy()
        with scene.materials_set_to(mats):
            paths = rt.compute_paths(ctx, scene, params, [tx], rxs)
            H = rt.paths_cfr(ctx, paths, params.freq_hz, **cfr_kw)
        fctx.rt = (ctx, scene, params, tx, rxs, cfr_kw, paths, mats)
        return H[0]

    @staticmethod
    def backward(fctx, G):
        ctx, scene, params, tx, rxs, cfr_kw, paths, mats = fctx.rt
        g = rt.paths_cfr_adjoint(ctx, paths, G[None], params.freq_hz, **cfr_kw)
        with scene.materials_set_to(mats):
            grad = rt.paths_coef_grad(ctx, scene, params, tx, rxs, paths["depth"][0], paths["faces"][0], g[0])
        return grad[:2 * scene.nm], None, None, None, None, None, None


def channel_frequency_response(theta, ctx, scene, params, tx, rxs, **cfr_kw):
    """Differentiable H of one transmitter (see rt.paths_cfr for cfr_kw)."""
    return ChannelFrequencyResponse.apply(theta, ctx, scene, params, tx, rxs, cfr_kw)
