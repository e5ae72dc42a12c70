"""GPU parity of diffusely scattered paths (rt_compute_scattering) with the
FP64 oracle (oracle/scatpaths.py): per receiver the (ray, depth) keys, their
order, coefficients, transfer matrices, delays, angles and faces; at full size
(2.5e6 rays, three chunks) on a lattice sample.  Also the specular share that
scattering coefficients give the paths of rt_compute_paths and their power
gradient (oracle/image.py, oracle/grad.py)."""
import copy

import numpy as np
import pytest
import torch

import scenegen as sg
from oracle import geom, grad as ograd, image, sbr, scatpaths

from gpu_common import ctx, lib, oracle_params, params, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]


def _scene_with(s, S):
    """A scene instance of its own (scattering coefficients are scene state)."""
    sc = lib().Scene.from_scenegen(ctx(), s)
    sc.set_scattering(S, 1)
    return sc


def _ambiguous_rays(s, tx, p, delta=1e-6):
    """Lattice indices of the rays that pass within delta of a triangle edge
    before their last scattering hit (the oracle and the GPU may route them
    differently)."""
    res = sbr.trace(s, tx, oracle_params(p), record=True)
    amb = np.zeros(res.ray_idx.shape[0], dtype=bool)
    for k in range(p.max_depth):
        amb |= res.margin[k] < delta
    return set(int(i) for i in res.ray_idx[amb])


def _angle_diff(x, y):
    d = np.abs(np.asarray(x, dtype=np.float64) - np.asarray(y, dtype=np.float64))
    return np.minimum(d, 2 * np.pi - d)


def _compare(o, ref, amb, t=0, keep=None):
    """Compares every receiver's GPU paths with the oracle's; ``keep(ray)``
    restricts the GPU side to the oracle's sample.  Returns (checked, excused)."""
    n = o["num_paths"][t].cpu().numpy()
    ray = o["ray"][t].cpu().numpy()
    depth = o["depth"][t].cpu().numpy()
    faces = o["faces"][t].cpu().numpy()
    a = o["a"][t].cpu().numpy()
    T = o["T"][t].cpu().numpy()
    tau = o["tau"][t].cpu().numpy()
    aod = o["aod"][t].cpu().numpy()
    aoa = o["aoa"][t].cpu().numpy()
    P = ray.shape[1]
    checked = excused = 0
    for r, pl in enumerate(ref):
        nr = int(n[r])
        assert nr <= P
        keys = list(zip(ray[r, :nr].tolist(), depth[r, :nr].tolist()))
        assert keys == sorted(keys) and len(set(keys)) == nr          # ordered by (ray, depth)
        assert np.all(depth[r, nr:] == -1) and np.all(ray[r, nr:] == -1) and np.all(tau[r, nr:] == -1.0)
        assert np.all(a[r, nr:] == 0.0)
        got = {k: j for j, k in enumerate(keys) if keep is None or keep(k[0])}
        want = {(p.ray, p.depth): p for p in pl}
        diff = set(got) ^ set(want)
        assert all(k[0] in amb for k in diff), ("rx %d" % r, sorted(set(got) - set(want))[:5],
                                                sorted(set(want) - set(got))[:5])
        excused += len(diff)
        for k in set(got) & set(want):
            j, p = got[k], want[k]
            ga = complex(a[r, j, 0], a[r, j, 1])
            assert abs(ga - p.a) <= 1e-4 * abs(p.a), (r, k, ga, p.a)
            Tg = T[r, j, ..., 0] + 1j * T[r, j, ..., 1]
            assert np.max(np.abs(Tg - p.T)) <= 1e-4 * np.max(np.abs(p.T)), (r, k)
            assert abs(tau[r, j] - p.tau) <= 1e-6 * p.tau
            assert np.max(_angle_diff(aod[r, j], p.aod)) < 1e-5
            assert np.max(_angle_diff(aoa[r, j], p.aoa)) < 1e-5
            fl = faces[r, j]
            assert tuple(int(f) for f in fl[:p.depth]) == p.faces and np.all(fl[p.depth:] == -1)
            checked += 1
    return checked, excused


def _case(case):
    if case == "toy":
        s = sg.make_toy()
        tx = sg.Device((-40.0, 5.0, 12.0))
        rxs = [sg.Device(q) for q in ((40.0, 0.0, 1.5), (0.0, 40.0, 3.0), (-60.0, -50.0, 2.0), (30.0, 30.0, 20.0),
                                      (0.0, 0.0, 20.0), (-20.0, -8.0, 1.5))]
        return s, tx, rxs, [0.7], 20_000, 2
    w = sg.urban_workload(num_rays=20_000) if case == "urban" else sg.diff_workload(num_rays=20_000)
    rxs = [copy.copy(r) for r in w.rx[:8]]
    tx = copy.copy(w.tx[0])
    if case == "urban_polarised":  # +45 degree TR 38.901 transmitter, H-pol dipole receivers
        tx.pol = sg.POL_SLANT_P45
        for r in rxs:
            r.pattern = sg.PATTERN_DIPOLE
            r.pol = sg.POL_H
            r.yaw = 0.7
    return w.scene, tx, rxs, [0.6, 0.35], 20_000, 3


@pytest.mark.parametrize("case", ["toy", "urban", "urban_polarised"])
def test_scattered_paths_match_oracle(case):
    m = lib()
    s, tx, rxs, S, N, D = _case(case)
    sc = _scene_with(s, S)
    p = m.TraceParams(freq_hz=s.freq_hz, max_depth=D, num_rays=N)
    o = m.compute_scattering(ctx(), sc, p, [tx], rxs, P=3 * N)
    ref = scatpaths.paths(s, tx, rxs, oracle_params(p), S)
    checked, excused = _compare(o, ref, _ambiguous_rays(s, tx, p))
    print("%s: %d paths compared, %d on ambiguous rays" % (case, checked, excused))
    assert checked > 200 * len(rxs) // 8 and excused <= 0.01 * checked


def test_full_size_three_chunks_on_a_lattice_sample():
    """2.5e6 rays (three chunks of 2^20), depth 3, two receivers: every path of
    the sampled rays equals the oracle's; the counts are the slots written."""
    m = lib()
    w = sg.urban_workload(num_rays=2_500_000)
    S = [0.6, 0.35]
    sc = _scene_with(w.scene, S)
    rxs = w.rx[:2]
    p = m.TraceParams(freq_hz=w.scene.freq_hz, max_depth=3, num_rays=w.num_rays)
    o = m.compute_scattering(ctx(), sc, p, w.tx, rxs, P=4_000_000)
    sub = m.TraceParams(freq_hz=w.scene.freq_hz, max_depth=3, num_rays=w.num_rays, ray_begin=11, ray_stride=997)
    ref = scatpaths.paths(w.scene, w.tx[0], rxs, oracle_params(sub), S)
    checked, excused = _compare(o, ref, _ambiguous_rays(w.scene, w.tx[0], sub), keep=lambda i: i % 997 == 11)
    n = o["num_paths"][0].cpu().numpy()
    print("full size: %s paths per receiver, %d sampled compared, %d excused" % (n.tolist(), checked, excused))
    assert n.min() > 50_000 and checked > 300 and excused <= 0.01 * checked


def test_capacity_and_arguments():
    m = lib()
    s, tx, rxs, S, N, D = _case("toy")
    sc = _scene_with(s, S)
    p = m.TraceParams(freq_hz=s.freq_hz, max_depth=D, num_rays=N)
    full = m.compute_scattering(ctx(), sc, p, [tx], rxs, P=3 * N)
    with pytest.raises(m._lib.RTError) as e:
        m.compute_scattering(ctx(), sc, p, [tx], rxs, P=5)
    assert e.value.code == m._lib.RT_ERR_CAPACITY
    with pytest.raises(m._lib.RTError) as e:
        m.compute_scattering(ctx(), sc, p, [tx], rxs, P=0)
    assert e.value.code == m._lib.RT_ERR_ARG
    # truncated output: the first P slots of the full result, true counts
    import ctypes
    L = m._lib
    P = 5
    o = {k: torch.empty((1, len(rxs), P) + sh, dtype=dt, device="cuda") for k, sh, dt in (
        ("a", (2,), torch.float32), ("T", (2, 2, 2), torch.float32), ("tau", (), torch.float32),
        ("aod", (2,), torch.float32), ("aoa", (2,), torch.float32), ("depth", (), torch.int32),
        ("ray", (), torch.int64), ("faces", (D,), torch.int32))}
    o["num_paths"] = torch.empty((1, len(rxs)), dtype=torch.int64, device="cuda")
    tx_arr = (L.rt_device * 1)(m.rt.device_struct(tx))
    rx_arr = (L.rt_device * len(rxs))(*[m.rt.device_struct(r) for r in rxs])
    pc = p.c()
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = L.lib.rt_compute_scattering(ctx().h, sc.h, ctypes.byref(pc), tx_arr, 1, rx_arr, len(rxs), P, ptr(o["a"]),
                                     ptr(o["T"]), ptr(o["tau"]), ptr(o["aod"]), ptr(o["aoa"]), ptr(o["depth"]),
                                     ptr(o["ray"]), ptr(o["faces"]), ptr(o["num_paths"]))
    assert rc == L.RT_ERR_CAPACITY
    torch.cuda.synchronize()
    assert torch.equal(o["num_paths"], full["num_paths"])
    for k in ("a", "T", "tau", "ray", "depth", "faces"):
        assert torch.equal(o[k], full[k][:, :, :P]), k
    # no scattering material, or depth 0: no paths
    sc0 = _scene_with(s, [0.0])
    o0 = m.compute_scattering(ctx(), sc0, p, [tx], rxs, P=4)
    assert int(o0["num_paths"].sum()) == 0 and bool((o0["depth"] == -1).all())
    p0 = m.TraceParams(freq_hz=s.freq_hz, max_depth=0, num_rays=N)
    assert int(m.compute_scattering(ctx(), sc, p0, [tx], rxs, P=4)["num_paths"].sum()) == 0


def _gpu_sequences(o, nrx):
    depth = o["depth"][0].cpu().numpy()
    faces = o["faces"][0].cpu().numpy()
    return [[tuple(int(f) for f in faces[r, j, :depth[r, j]]) for j in range(depth.shape[1]) if depth[r, j] >= 0]
            for r in range(nrx)]


def test_specular_paths_keep_their_share_with_scattering():
    m = lib()
    w = sg.diff_workload()      # 1e6 rays, depth 3, 256 receivers
    S = [0.6, 0.35]
    sc = _scene_with(w.scene, S)
    p = params(w, max_paths_per_rx=64)
    o = m.compute_paths(ctx(), sc, p, w.tx, w.rx)
    g = geom.Geometry(w.scene)
    seqs = _gpu_sequences(o, len(w.rx))
    n = o["num_paths"][0].cpu().numpy()
    a = o["a"][0].cpu().numpy()
    checked = 0
    shared = 0
    for r in range(len(w.rx)):
        want = {q.faces: q for q in image.paths(g, w.tx[0], [w.rx[r]], seqs[r], scat=S)[0]}
        for j in range(int(n[r])):
            q = want[seqs[r][j]]
            ga = complex(a[r, j, 0], a[r, j, 1])
            assert abs(ga - q.a) <= 1e-4 * abs(q.a), (r, seqs[r][j], ga, q.a)
            checked += 1
            shared += image.specular_share(g, seqs[r][j], S) < 1.0
    assert checked > 100 and shared > 50


def test_power_gradient_with_scattering_matches_central_differences():
    lib()
    from paper_2303_11103_amd.autograd import received_power
    w = sg.diff_workload(num_rays=100_000)
    w.rx = w.rx[:40]
    S = [0.6, 0.35]
    sc = _scene_with(w.scene, S)
    p = params(w, max_paths_per_rx=64)
    tx = w.tx[0]
    theta = torch.tensor(list(np.asarray(w.scene.materials, dtype=np.float64).reshape(-1)) + list(tx.pos) +
                         [tx.yaw, tx.pitch], dtype=torch.float64, device="cuda", requires_grad=True)
    P = received_power(theta, ctx(), sc, p, tx, w.rx)
    used = P > 0
    L = torch.mean(10 * torch.log10(P[used]))
    L.backward()
    o = lib().compute_paths(ctx(), sc, p, w.tx, w.rx)
    g = geom.Geometry(w.scene)
    fd, _, unstable = ograd.fd_gradient(g, tx, w.rx, _gpu_sequences(o, len(w.rx)), mask=used.cpu().numpy(), scat=S)
    assert not unstable.any()
    gg = theta.grad.cpu().numpy()
    scale = np.abs(fd)
    big = scale > 1e-6 * scale.max()
    assert np.max(np.abs(gg - fd)[big] / scale[big]) < 1e-3, (gg, fd)


def test_channel_response_over_specular_diffracted_and_scattered_paths():
    """combine_paths + rt_paths_cfr: the response of the combined list equals
    the oracle's response of the same paths and the sum of the three kinds'
    responses."""
    from oracle import channel
    m = lib()
    s, tx, rxs, S, N, D = _case("toy")
    rxs = rxs[:3]
    sc = _scene_with(s, S)
    p = m.TraceParams(freq_hz=s.freq_hz, max_depth=D, num_rays=N, max_paths_per_rx=32)
    spec = m.compute_paths(ctx(), sc, p, [tx], rxs)
    diff = m.compute_diffraction(ctx(), sc, s.freq_hz, [tx], rxs, P=32)
    ps = m.TraceParams(freq_hz=s.freq_hz, max_depth=D, num_rays=5000)
    scat = m.compute_scattering(ctx(), sc, ps, [tx], rxs, P=12_000)
    comb = m.combine_paths(spec, diff, scat)
    kw = dict(num_subcarriers=32, spacing=30e3)
    H = m.paths_cfr(ctx(), comb, s.freq_hz, **kw)
    parts = sum(m.paths_cfr(ctx(), q, s.freq_hz, **kw) for q in (spec, m.combine_paths(diff), scat))
    a = comb["a"][0].cpu().numpy()
    tau = comb["tau"][0].cpu().numpy()
    aod = comb["aod"][0].cpu().numpy()
    aoa = comb["aoa"][0].cpu().numpy()
    depth = comb["depth"][0].cpu().numpy()
    Hn = H.cpu().numpy()
    kinds = [0, 0, 0]
    for r in range(len(rxs)):
        pl = [(complex(a[r, j, 0], a[r, j, 1]), float(tau[r, j]), tuple(aod[r, j].astype(float)),
               tuple(aoa[r, j].astype(float))) for j in range(a.shape[1]) if depth[r, j] >= 0]
        scale = sum(abs(x[0]) for x in pl)
        ref = channel.cfr(pl, s.freq_hz, 32, 30e3)
        assert np.max(np.abs(Hn[0, r] - ref)) <= 1e-5 * scale, r
        assert torch.max(torch.abs(H[0, r] - parts[0, r])).item() <= 1e-5 * scale
        for k, q in enumerate((spec["depth"], diff["wedge"], scat["depth"])):
            kinds[k] += int((q[0, r] >= 0).sum())
    assert min(kinds) > 0, kinds


def test_two_transmitters_equal_separate_calls():
    m = lib()
    s, tx, rxs, S, N, D = _case("toy")
    tx2 = sg.Device((35.0, -30.0, 8.0), pattern=sg.PATTERN_TR38901, yaw=2.5, pol=sg.POL_SLANT_M45)
    sc = _scene_with(s, S)
    p = m.TraceParams(freq_hz=s.freq_hz, max_depth=D, num_rays=8000)
    both = m.compute_scattering(ctx(), sc, p, [tx, tx2], rxs, P=20_000)
    for t, one in enumerate((tx, tx2)):
        single = m.compute_scattering(ctx(), sc, p, [one], rxs, P=20_000)
        for k in ("a", "T", "tau", "aod", "aoa", "depth", "ray", "faces", "num_paths"):
            assert torch.equal(both[k][t], single[k][0]), (t, k)
    assert int(both["num_paths"][1].sum()) > 1000
