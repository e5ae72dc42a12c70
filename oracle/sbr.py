"""Shoot-and-bounce tracing and the coverage-map estimator (float64).

Test infrastructure: see the package docstring.

Paper Sec. II-B: rays leave the transmitter in Fibonacci-lattice directions and
propagate through the scene, reflecting specularly, until the maximum number
of reflections is reached; Sec. II-A: a coverage map gives the path gain per
cell of a plane.  The paper gives no estimator; the one used here follows from
ray tubes:

* every ray carries the solid angle 4 pi / N; its tube cross-section at
  distance s is s^2 4 pi / N, its footprint on a horizontal plane that area
  divided by |d_z|;
* averaging the received power of a receiver with field pattern F_rx over a
  cell of area A gives, per crossing of the plane z = z_grid by a segment,
      dg = (lambda / 4 pi)^2 (4 pi / N) |F_rx(-d) . E|^2 / (A |d_z|),
  where E starts as the transmitter field F_tx(d_0) and is multiplied by the
  reflection operator at every bounce (the 1/s^2 spreading cancels);
* a segment from o with direction d and hit distance t_hit (inf on a miss)
  crosses the plane at t_c = (z - o_z)/d_z when |d_z| >= 1e-12 and
  0 < t_c < t_hit; the cell is (floor((x - x0)/cell), floor((y - y0)/cell)),
  crossings outside the grid are dropped; every crossing adds one hit.

Depth semantics: max_depth D is the maximum number of reflections (D = 0 is
line of sight only), so a ray traces at most D + 1 segments.  The paper's
sentence that depth one gives only LOS conflicts with its own definition of
max_depth as the number of interactions; the definition is used.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import em, fib, native, scatter as scat
from .consts import TMIN_DEFAULT
from .geom import Geometry


@dataclass
class TraceParams:
    num_rays: int
    max_depth: int
    tmin: float = TMIN_DEFAULT
    ray_begin: int = 0
    ray_stride: int = 1


@dataclass
class TraceResult:
    ray_idx: np.ndarray                       # traced ray indices
    hit_tri: list = field(default_factory=list)   # per segment k: tri id per ray (-1 miss, -2 dead)
    hit_t: list = field(default_factory=list)
    margin: list = field(default_factory=list)    # per segment k: edge margin per ray (inf when dead)
    origins: list = field(default_factory=list)   # per segment k: float64 origins (nan when dead)
    dirs: list = field(default_factory=list)
    gain: np.ndarray = None                   # (ny, nx) linear path gain
    hits: np.ndarray = None                   # (ny, nx) crossings
    ambiguous: np.ndarray = None              # per ray: passed within delta of an edge / cell border
    cell_rays: list = None                    # per crossing: (ray position, flat cell)
    candidates: set = None                    # face sequences (tuples) of every hit prefix


def _cross_plane(o, d, t_hit, grid):
    dz = d[:, 2]
    ok = np.abs(dz) >= 1e-12
    with np.errstate(divide="ignore", invalid="ignore"):
        tc = np.where(ok, (grid.z - o[:, 2]) / np.where(ok, dz, 1.0), -1.0)
    ok &= (tc > 0.0) & (tc < t_hit)
    x = o[:, 0] + tc * d[:, 0]
    y = o[:, 1] + tc * d[:, 1]
    fx = (x - grid.x0) / grid.cell
    fy = (y - grid.y0) / grid.cell
    ix = np.floor(fx)
    iy = np.floor(fy)
    ok &= (ix >= 0) & (ix < grid.nx) & (iy >= 0) & (iy < grid.ny)
    return ok, ix, iy, fx, fy, tc


def trace(scene, tx, params: TraceParams, grid=None, rx_ant=None, record=False, delta=1e-6,
          candidates=False, threads=None, geo=None, idx=None, sphere=None, scattering=None) -> TraceResult:
    """Trace the (sub)set of lattice rays of one transmitter.

    With ``grid`` the coverage map (gain, hits) is accumulated; ``record``
    keeps per-segment hits, origins and directions; ``candidates`` collects the
    face sequence of every hit prefix of length 1..max_depth.  ``idx``
    (optional) lists the lattice indices to trace instead of the params'
    sub-lattice.

    ``sphere = (rx_positions [nrx][3], kappa)`` collects reception-sphere
    candidates: the sequence of the reflections before a segment becomes a
    candidate of receiver R when the segment's closest approach to R, at
    t* = clamp((R - o) . d, 0, t_hit), lies within kappa (s + t*) sqrt(4 pi / n)
    of R (s the path length before the segment, n the number of traced rays):
    ``res.sphere_pairs[r]`` is the set of sequences of receiver r,
    ``res.sphere_sure[r]`` those accepted by a ray that never passed within
    delta of an edge, away from the radius, and ``res.sphere_borderline`` the
    (r, sequence) pairs decided within 1e-6 relative of the radius by some ray.

    ``scattering = (S [nm], seed)`` makes reflections diffuse with probability
    S^2 of the hit material (Lambertian, see oracle.scatter).
    """
    geo = geo or Geometry(scene)
    lam = em.wavelength(geo.freq)
    N = int(params.num_rays)
    idx = fib.subset(N, params.ray_begin, params.ray_stride) if idx is None else np.asarray(idx, dtype=np.int64)
    n = idx.shape[0]
    d = fib.directions(N, idx)
    o = np.repeat(np.asarray(tx.pos, dtype=np.float64)[None, :], n, axis=0)
    E = em.antenna_field(tx, d).astype(np.complex128)
    excl = np.full(n, -1, dtype=np.int32)
    alive = np.arange(n)
    res = TraceResult(ray_idx=idx)
    res.ambiguous = np.zeros(n, dtype=bool)
    if grid is not None:
        gain = np.zeros(grid.ny * grid.nx, dtype=np.float64)
        hits = np.zeros(grid.ny * grid.nx, dtype=np.int64)
        cell_ray = []
        scale = (lam / (4.0 * np.pi)) ** 2 * (4.0 * np.pi / N) / (grid.cell * grid.cell)
        rx_ant = rx_ant or _iso()
    seqs = [() for _ in range(n)] if (candidates or sphere is not None) else None
    cand = set() if candidates else None
    if sphere is not None:
        rx_pos = np.asarray(sphere[0], dtype=np.float64).reshape(-1, 3)
        sk = float(sphere[1]) * np.sqrt(4.0 * np.pi / n)
        path_len = np.zeros(n)
        res.sphere_pairs = [set() for _ in range(rx_pos.shape[0])]
        res.sphere_sure = [set() for _ in range(rx_pos.shape[0])]
        res.sphere_borderline = set()
    eta_m = em.eta(geo.materials[:, 0], geo.materials[:, 1], geo.freq)
    pec_m = ~np.isfinite(geo.materials[:, 1])

    for k in range(params.max_depth + 1):
        if alive.size == 0:
            if record:
                res.hit_tri.append(np.full(n, -2, dtype=np.int32))
                res.hit_t.append(np.full(n, np.inf))
                res.margin.append(np.full(n, np.inf))
                res.origins.append(np.full((n, 3), np.nan))
                res.dirs.append(np.full((n, 3), np.nan))
            continue
        tri, t, margin = native.closest_hit(o, d, excl, params.tmin, geo.V, geo.F, geo.face,
                                            want_margin=True, threads=threads)
        res.ambiguous[alive] |= margin < delta
        if record:
            full_tri = np.full(n, -2, dtype=np.int32)
            full_tri[alive] = tri
            full_t = np.full(n, np.inf)
            full_t[alive] = t
            full_m = np.full(n, np.inf)
            full_m[alive] = margin
            fo = np.full((n, 3), np.nan)
            fo[alive] = o
            fd = np.full((n, 3), np.nan)
            fd[alive] = d
            res.hit_tri.append(full_tri)
            res.hit_t.append(full_t)
            res.margin.append(full_m)
            res.origins.append(fo)
            res.dirs.append(fd)
        if grid is not None:
            ok, ix, iy, fx, fy, tc = _cross_plane(o, d, t, grid)
            frx = em.antenna_field(rx_ant, -d)
            amp = np.einsum("ij,ij->i", frx.astype(np.complex128), E)
            w = scale * np.abs(amp) ** 2 / np.abs(d[:, 2])
            cell = (iy * grid.nx + ix)
            sel = np.nonzero(ok)[0]
            c = cell[sel].astype(np.int64)
            np.add.at(gain, c, w[sel])
            np.add.at(hits, c, 1)
            cell_ray.append(np.stack([alive[sel], c], axis=1))
            # a crossing is borderline when it lies within delta of a cell border
            # (grid boundary included), of the segment's origin or of its hit point
            dz = d[:, 2]
            valid = np.abs(dz) >= 1e-12
            with np.errstate(divide="ignore", invalid="ignore"):
                tcu = np.where(valid, (grid.z - o[:, 2]) / np.where(valid, dz, 1.0), -np.inf)
            xu = o[:, 0] + tcu * d[:, 0]
            yu = o[:, 1] + tcu * d[:, 1]
            fxu = (xu - grid.x0) / grid.cell
            fyu = (yu - grid.y0) / grid.cell
            border = np.minimum(np.abs(fxu - np.rint(fxu)), np.abs(fyu - np.rint(fyu))) * grid.cell < delta
            span = valid & (tcu > -delta) & (tcu < t + delta)
            borderline = span & (border | (np.abs(tcu) < delta) | (np.abs(tcu - t) < delta))
            res.ambiguous[alive[borderline]] = True
        if sphere is not None and k >= 1:
            _sphere_pairs(res, rx_pos, sk, o, d, t, path_len[alive], [seqs[r] for r in alive], res.ambiguous[alive])
        if k == params.max_depth:
            break
        hit = tri >= 0
        alive, o, d, E, tri, t = alive[hit], o[hit], d[hit], E[hit], tri[hit], t[hit]
        if alive.size == 0:
            continue
        p = o + t[:, None] * d
        n_tri = geo.normal[tri]
        d_r, n_f, cos_i = em.reflect(d, n_tri)
        m = geo.tri_mat[tri]
        r_perp, r_par = em.fresnel(eta_m[m], cos_i, pec=pec_m[m])
        if scattering is not None:
            S = np.asarray(scattering[0], dtype=np.float32).astype(np.float64)[m]
            ray_i = idx[alive]
            u = scat.uniform(scattering[1], scat.counter(ray_i, k, params.max_depth, 0))
            dif = u < S * S
            if np.any(dif):
                u1 = scat.uniform(scattering[1], scat.counter(ray_i[dif], k, params.max_depth, 1))
                u2 = scat.uniform(scattering[1], scat.counter(ray_i[dif], k, params.max_depth, 2))
                d_s = d_r.copy()
                d_s[dif] = scat.lambert_dirs(n_f[dif], u1, u2)
                E_s = em.transfer(E, d, d_r, n_f, r_perp, r_par)
                E_s[dif] = em.transfer_scattered(E[dif], d[dif], d_s[dif], n_f[dif], r_perp[dif], r_par[dif])
                E, d_r = E_s, d_s
            else:
                E = em.transfer(E, d, d_r, n_f, r_perp, r_par)
        else:
            E = em.transfer(E, d, d_r, n_f, r_perp, r_par)
        o, d = p, d_r
        excl = geo.face[tri].astype(np.int32)
        if sphere is not None:
            path_len[alive] += t
        if seqs is not None:
            for j, r in enumerate(alive):
                s = seqs[r] + (int(excl[j]),)
                seqs[r] = s
                if candidates:
                    cand.add(s)
    if grid is not None:
        res.gain = gain.reshape(grid.ny, grid.nx)
        res.hits = hits.reshape(grid.ny, grid.nx)
        res.cell_rays = cell_ray
    res.candidates = cand
    return res


def _sphere_pairs(res, R, sk, o, d, t, s_len, seq, amb_ray, chunk=4096):
    """Receiver spheres passed by the segments o + t' d, 0 <= t' <= t.  A pair
    is also "sure" when a ray that never came within delta of an edge accepted
    it away from the radius."""
    for c0 in range(0, o.shape[0], chunk):
        oo, dd, tt, ss = o[c0:c0 + chunk], d[c0:c0 + chunk], t[c0:c0 + chunk], s_len[c0:c0 + chunk]
        w = R[None, :, :] - oo[:, None, :]
        ts = np.einsum("mrk,mk->mr", w, dd)
        ts = np.minimum(np.maximum(ts, 0.0), tt[:, None])
        q = oo[:, None, :] + ts[..., None] * dd[:, None, :] - R[None, :, :]
        dist = np.sqrt(np.einsum("mrk,mrk->mr", q, q))
        rad = sk * (ss[:, None] + ts)
        acc = dist <= rad
        border = np.abs(dist - rad) <= 1e-6 * rad
        for mi, ri in zip(*np.nonzero(acc | border)):
            sq = seq[c0 + mi]
            if acc[mi, ri]:
                res.sphere_pairs[ri].add(sq)
                if not border[mi, ri] and not amb_ray[c0 + mi]:
                    res.sphere_sure[ri].add(sq)
            if border[mi, ri]:
                res.sphere_borderline.add((int(ri), sq))


def _iso():
    from types import SimpleNamespace
    return SimpleNamespace(yaw=0.0, pitch=0.0, roll=0.0, pattern=em.PATTERN_ISO)


def coverage(scene, tx, params, grid, rx_ant=None, threads=None, geo=None, delta=1e-6, scattering=None):
    """(gain (ny, nx), hits (ny, nx), number of ambiguous rays) for one
    transmitter.  A ray is ambiguous when it passes within ``delta`` of a
    triangle edge it could hit, or crosses the grid plane within ``delta`` of
    a cell border, of its origin or of its hit point; an implementation that
    rounds differently may route such a ray differently, which changes at most
    2 (max_depth + 1) cells per ambiguous ray."""
    r = trace(scene, tx, params, grid=grid, rx_ant=rx_ant, threads=threads, geo=geo, delta=delta,
              scattering=scattering)
    return r.gain, r.hits, int(r.ambiguous.sum())


def to_db(gain):
    with np.errstate(divide="ignore"):
        return 10.0 * np.log10(gain)
