"""Coverage-map gradient (rt_coverage_grad): the region's summed path gain and
its derivatives with respect to the materials and the transmitter yaw and
pitch, from a replay of the recorded rays with field tangents, against the
FP64 oracle's region gain and its central differences; the autograd Function
around it; and gradient ascent on the transmitter orientation for the
coverage of a region (the coverage counterpart of the orientation
optimisation of Sec. III-B)."""
import numpy as np
import pytest
import torch

import scenegen as sg
from oracle import covgrad

from gpu_common import ctx, lib, oracle_params, params, requires_gpu, scene

pytestmark = [pytest.mark.gpu, requires_gpu]

GRID = sg.Grid(-200.0, -200.0, 4.0, 100, 100, 1.5)


def _region(x0, x1, y0, y1):
    r = np.zeros((GRID.ny, GRID.nx), dtype=np.uint8)
    xs = GRID.x0 + (np.arange(GRID.nx) + 0.5) * GRID.cell
    ys = GRID.y0 + (np.arange(GRID.ny) + 0.5) * GRID.cell
    r[np.ix_((ys >= y0) & (ys < y1), (xs >= x0) & (xs < x1))] = 1
    return r


def _gpu(m, sc, p, tx, region):
    tri, t = m.trace_record(ctx(), sc, p, tx)
    reg = None if region is None else torch.from_numpy(region).to(ctx().torch_device)
    return m.coverage_grad(ctx(), sc, p, tx, GRID, tri, t, region=reg).cpu().numpy()


@pytest.mark.parametrize("region_box", [None, (-150.0, 0.0, -60.0, 90.0)])
def test_coverage_gradient_matches_oracle_central_differences(region_box):
    m = lib()
    w = sg.diff_workload(num_rays=100_000)
    p = params(w)
    sc = scene(w.scene)
    region = None if region_box is None else _region(*region_box)
    out = _gpu(m, sc, p, w.tx[0], region)
    G_ref, g_ref = covgrad.region_gain_fd(w.scene, w.tx[0], oracle_params(p), GRID, region=region)
    print("G gpu %.9e oracle %.9e" % (out[0], G_ref), flush=True)
    # the same rays: rays that pass within 1e-6 m of an edge may take other faces
    assert abs(out[0] - G_ref) < 1e-4 * G_ref
    # the replay agrees with the forward kernel's own (fp32) map
    cov = m.coverage_map(ctx(), sc, p, w.tx[0], GRID)
    gain = cov["gain"].double().cpu().numpy()
    G_fwd = gain.sum() if region is None else gain[region != 0].sum()
    assert abs(out[0] - G_fwd) < 1e-4 * G_fwd
    g = out[1:]
    scale = np.abs(g_ref)
    big = scale > 1e-6 * scale.max()
    err = np.abs(g - g_ref)[big] / scale[big]
    print("gradient gpu", g, "\noracle fd   ", g_ref, "\nrel", err, flush=True)
    assert err.max() < 1e-3


def test_autograd_function_and_orientation_ascent_for_a_region():
    m = lib()
    from paper_2303_11103_amd.autograd import coverage_region_gain
    w = sg.diff_workload(num_rays=100_000)
    p = params(w)
    sc = scene(w.scene)
    tx = w.tx[0]
    region = _region(-150.0, -50.0, 50.0, 150.0)   # behind and to the side of the boresight
    reg = torch.from_numpy(region).to(ctx().torch_device)
    mats = np.asarray(w.scene.materials, dtype=np.float64)
    try:
        theta = torch.tensor(list(mats.reshape(-1)) + [tx.yaw, tx.pitch], dtype=torch.float64,
                             device=ctx().torch_device, requires_grad=True)
        G = coverage_region_gain(theta, ctx(), sc, p, tx, GRID, reg)
        G.backward()
        direct = _gpu(m, sc, p, tx, region)
        assert abs(float(G) - direct[0]) <= 1e-12 * direct[0]
        assert np.allclose(theta.grad.cpu().numpy(), direct[1:], rtol=1e-12, atol=0.0)
        # normalised gradient ascent on (yaw, pitch) with backtracking: a step
        # that lowers the region gain is undone and the step halved
        def gain_and_grad(ang):
            th = torch.cat([torch.tensor(mats.reshape(-1), dtype=torch.float64), ang]).to(ctx().torch_device)
            th.requires_grad_(True)
            Gk = coverage_region_gain(th, ctx(), sc, p, tx, GRID, reg)
            Gk.backward()
            return float(Gk), th.grad[-2:].cpu()

        ang = torch.tensor([tx.yaw, tx.pitch], dtype=torch.float64)
        G0, d = gain_and_grad(ang)
        accepted, step = [G0], 0.2
        for _ in range(12):
            trial = ang + step * d / d.norm()
            Gt, dt = gain_and_grad(trial)
            if Gt > accepted[-1]:
                ang, d = trial, dt
                accepted.append(Gt)
            else:
                step *= 0.5
        print("accepted region gains", accepted, "final yaw/pitch", ang.tolist(), flush=True)
        assert len(accepted) >= 3
        assert accepted[-1] > 1.15 * accepted[0]
    finally:
        sc.set_materials(mats)


def test_coverage_grad_argument_errors():
    m = lib()
    w = sg.diff_workload(num_rays=10_000)
    p = params(w)
    sc = scene(w.scene)
    tri, t = m.trace_record(ctx(), sc, p, w.tx[0])
    with pytest.raises(ValueError):
        m.coverage_grad(ctx(), sc, p, w.tx[0], GRID, tri[:, :5], t[:, :5])
    with pytest.raises(ValueError):
        m.coverage_grad(ctx(), sc, p, w.tx[0], GRID, tri, t,
                        region=torch.ones((3, 3), dtype=torch.uint8, device=ctx().torch_device))
    s5 = sg.make_urban(0)
    s5.tri_mat = (np.arange(s5.nt) % 5).astype(np.int32)
    s5.materials = np.tile(np.asarray(s5.materials[:1]), (5, 1))
    s5.material_names = ["m%d" % i for i in range(5)]
    sc5 = m.Scene.from_scenegen(ctx(), s5)
    tri5, t5 = m.trace_record(ctx(), sc5, p, w.tx[0])
    with pytest.raises(RuntimeError, match="at most 4 materials"):
        m.coverage_grad(ctx(), sc5, p, w.tx[0], GRID, tri5, t5)


def test_coverage_gradient_of_sub_lattices_adds_up_and_empty_region_is_zero():
    m = lib()
    w = sg.diff_workload(num_rays=60_000)
    sc = scene(w.scene)
    full = _gpu(m, sc, params(w), w.tx[0], None)
    parts = sum(_gpu(m, sc, params(w, ray_begin=b, ray_stride=3), w.tx[0], None) for b in range(3))
    assert np.allclose(parts, full, rtol=1e-9, atol=1e-12 * np.abs(full).max())
    zero = _gpu(m, sc, params(w), w.tx[0], np.zeros((GRID.ny, GRID.nx), dtype=np.uint8))
    assert np.all(zero == 0.0)
