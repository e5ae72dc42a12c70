"""Seeded synthetic workloads: triangle-mesh scenes, radio devices and grids.

This module builds the inputs that both the FP64 oracle and the GPU library
consume.  It holds geometry construction and random draws only -- none of the
propagation arithmetic (no intersection, reflection, Fresnel or antenna math).

The paper's own scenes (OpenStreetMap extracts, Sec. II and III) are not
available; these procedural scenes stand in for them:

* ``make_toy``   -- ground quad plus one box building (14 triangles).
* ``make_urban`` -- 8x8 grid of box buildings, 40 m footprints, 20 m streets,
  heights U(10, 60) m, concrete or glass per building (770 triangles).
* ``make_city``  -- 50x50 blocks of extruded random convex polygons (2x2 lots
  per block), log-normal heights, concrete/glass/metal (about 220k triangles).

Radio materials are given as (relative permittivity, conductivity S/m) at the
carrier frequency; the paper characterises a material by exactly this pair
with unit relative permeability (Sec. II) and takes frequency-dependent values
from the ITU-R P.2040 model, whose values at 3.5 GHz and 28 GHz are listed in
``MATERIALS_3P5GHZ`` and ``MATERIALS_28GHZ``.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

# (eps_r, sigma [S/m]) per material at the carrier.  ITU-R P.2040 model
# eps_r = a f^b, sigma = c f^d (f in GHz): concrete (5.31, 0, 0.0326, 0.8095),
# glass (6.27, 0, 0.0043, 1.1925), metal (1, 0, 1e7, 0).
MATERIALS_3P5GHZ = {"concrete": (5.31, 0.09), "glass": (6.27, 0.019)}
MATERIALS_28GHZ = {"concrete": (5.31, 0.4838), "glass": (6.27, 0.2290), "metal": (1.0, 1.0e7)}

PATTERN_ISO = 0
PATTERN_TR38901 = 1
PATTERN_DIPOLE = 2
POL_V, POL_H, POL_SLANT_P45, POL_SLANT_M45 = 0, 1, 2, 3


@dataclass
class Scene:
    name: str
    V: np.ndarray          # (nv, 3) float32 vertex positions [m]
    F: np.ndarray          # (nt, 3) int32 vertex indices per triangle
    tri_mat: np.ndarray    # (nt,) int32 material id per triangle
    materials: np.ndarray  # (nm, 2) float32: eps_r, sigma [S/m]
    material_names: list
    freq_hz: float
    footprints: list = field(default_factory=list)  # building footprints for rx sampling
    roofs: list = field(default_factory=list)       # (x, y, roof height, footprint area)

    @property
    def nt(self) -> int:
        return int(self.F.shape[0])

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.V, self.F, self.tri_mat, self.materials):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()[:16]


@dataclass
class Device:
    """A transmitter or receiver: position, orientation (yaw, pitch, roll in
    radians) and a single-element antenna (pattern id, vertical polarization)."""
    pos: tuple
    yaw: float = 0.0
    pitch: float = 0.0
    roll: float = 0.0
    pattern: int = PATTERN_ISO
    pol: int = 0


@dataclass
class Grid:
    """Horizontal coverage-map grid: cell (ix, iy) covers
    [x0 + ix*cell, x0 + (ix+1)*cell) x [y0 + iy*cell, y0 + (iy+1)*cell) at height z."""
    x0: float
    y0: float
    cell: float
    nx: int
    ny: int
    z: float


@dataclass
class Workload:
    scene: Scene
    tx: list
    rx: list
    grid: Grid
    num_rays: int
    max_depth: int
    rx_ant: Device = field(default_factory=lambda: Device(pos=(0.0, 0.0, 0.0)))


class _Mesh:
    def __init__(self):
        self.V = []
        self.F = []
        self.M = []

    def poly(self, pts, mat):
        """Append a planar convex polygon as a fan of triangles that all share
        the polygon's first vertex."""
        base = len(self.V)
        self.V.extend(pts)
        for k in range(1, len(pts) - 1):
            self.F.append((base, base + k, base + k + 1))
            self.M.append(mat)

    def box(self, x0, x1, y0, y1, z0, z1, mat):
        self.poly([(x0, y0, z0), (x1, y0, z0), (x1, y1, z0), (x0, y1, z0)], mat)  # floor
        self.poly([(x0, y0, z1), (x1, y0, z1), (x1, y1, z1), (x0, y1, z1)], mat)  # roof
        self.poly([(x0, y0, z0), (x1, y0, z0), (x1, y0, z1), (x0, y0, z1)], mat)
        self.poly([(x1, y0, z0), (x1, y1, z0), (x1, y1, z1), (x1, y0, z1)], mat)
        self.poly([(x1, y1, z0), (x0, y1, z0), (x0, y1, z1), (x1, y1, z1)], mat)
        self.poly([(x0, y1, z0), (x0, y0, z0), (x0, y0, z1), (x0, y1, z1)], mat)

    def arrays(self):
        return (np.asarray(self.V, dtype=np.float32).reshape(-1, 3),
                np.asarray(self.F, dtype=np.int32).reshape(-1, 3),
                np.asarray(self.M, dtype=np.int32))


def _mats(table, names):
    return np.asarray([table[n] for n in names], dtype=np.float32)


def make_toy() -> Scene:
    """200x200 m ground (2 triangles) plus a 20x10x15 m box (12 triangles),
    all concrete, 3.5 GHz."""
    m = _Mesh()
    m.poly([(-100, -100, 0), (100, -100, 0), (100, 100, 0), (-100, 100, 0)], 0)
    m.box(30, 50, -5, 5, 0, 15, 0)
    V, F, M = m.arrays()
    return Scene("toy", V, F, M, _mats(MATERIALS_3P5GHZ, ["concrete"]), ["concrete"], 3.5e9,
                 footprints=[(30.0, 50.0, -5.0, 5.0)], roofs=[(40.0, 0.0, 15.0, 200.0)])


def make_urban(seed: int = 0) -> Scene:
    """8x8 box buildings, 40x40 m footprints on a 60 m pitch centred at the
    origin, heights U(10, 60) m, concrete or glass with probability 1/2 each,
    on a [-300, 300]^2 concrete ground; 770 triangles, 3.5 GHz."""
    rng = np.random.default_rng(seed)
    heights = rng.uniform(10.0, 60.0, size=(8, 8))
    mats = rng.integers(0, 2, size=(8, 8))
    m = _Mesh()
    m.poly([(-300, -300, 0), (300, -300, 0), (300, 300, 0), (-300, 300, 0)], 0)
    fps, roofs = [], []
    for i in range(8):
        for j in range(8):
            cx, cy = -210.0 + 60.0 * i, -210.0 + 60.0 * j
            h = float(np.float32(heights[i, j]))
            m.box(cx - 20, cx + 20, cy - 20, cy + 20, 0.0, h, int(mats[i, j]))
            fps.append((cx - 20, cx + 20, cy - 20, cy + 20))
            roofs.append((cx, cy, h, 1600.0))
    V, F, M = m.arrays()
    return Scene("urban", V, F, M, _mats(MATERIALS_3P5GHZ, ["concrete", "glass"]),
                 ["concrete", "glass"], 3.5e9, footprints=fps, roofs=roofs)


def make_city(seed: int = 0, blocks: int = 50) -> Scene:
    """blocks x blocks city blocks on a 40 m pitch (30 m block, 10 m street)
    centred at the origin; 2x2 lots of 15 m per block, each holding one convex
    polygon of n ~ U{5..8} vertices at sorted uniform angles on a circle of
    radius U(4, 7) m, randomly rotated, extruded to a log-normal height
    (median 25 m, log-sd 0.5).  Materials per building uniform over
    concrete/glass/metal at 28 GHz; concrete ground."""
    rng = np.random.default_rng(seed)
    half = 20.0 * blocks
    m = _Mesh()
    m.poly([(-half, -half, 0), (half, -half, 0), (half, half, 0), (-half, half, 0)], 0)
    fps, roofs = [], []
    for bi in range(blocks):
        for bj in range(blocks):
            bx, by = -half + 40.0 * bi + 5.0, -half + 40.0 * bj + 5.0
            for li in range(2):
                for lj in range(2):
                    cx, cy = bx + 7.5 + 15.0 * li, by + 7.5 + 15.0 * lj
                    n = int(rng.integers(5, 9))
                    ang = np.sort(rng.uniform(0.0, 2 * np.pi, size=n)) + rng.uniform(0, 2 * np.pi)
                    r = rng.uniform(4.0, 7.0)
                    h = float(np.float32(rng.lognormal(np.log(25.0), 0.5)))
                    mat = int(rng.integers(0, 3))
                    px = (cx + r * np.cos(ang)).astype(np.float32)
                    py = (cy + r * np.sin(ang)).astype(np.float32)
                    pts = list(zip(px.tolist(), py.tolist()))
                    for k in range(n):
                        (ax, ay), (qx, qy) = pts[k], pts[(k + 1) % n]
                        m.poly([(ax, ay, 0.0), (qx, qy, 0.0), (qx, qy, h), (ax, ay, h)], mat)
                    m.poly([(x, y, h) for (x, y) in pts], mat)
                    m.poly([(x, y, 0.0) for (x, y) in pts[::-1]], mat)
                    area = 0.5 * abs(float(np.dot(px, np.roll(py, -1)) - np.dot(py, np.roll(px, -1))))
                    fps.append((float(px.min()), float(px.max()), float(py.min()), float(py.max())))
                    roofs.append((float(px.mean()), float(py.mean()), h, area))
    V, F, M = m.arrays()
    names = ["concrete", "glass", "metal"]
    return Scene("city", V, F, M, _mats(MATERIALS_28GHZ, names), names, 28e9,
                 footprints=fps, roofs=roofs)


def _inside_any(x, y, fps, margin):
    for (x0, x1, y0, y1) in fps:
        if x0 - margin <= x <= x1 + margin and y0 - margin <= y <= y1 + margin:
            return True
    return False


def sample_street_points(scene: Scene, n: int, lo: float, hi: float, z: float, seed: int,
                         margin: float = 1.0) -> np.ndarray:
    """n points uniform in [lo, hi]^2 at height z that lie outside every
    building footprint (expanded by margin), by rejection."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        x, y = rng.uniform(lo, hi, size=2)
        if not _inside_any(x, y, scene.footprints, margin):
            out.append((x, y, z))
    return np.asarray(out, dtype=np.float32)


def _city_street_points(n, half, z, seed):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        x, y = rng.uniform(-half, half, size=2)
        fx, fy = (x + half) % 40.0, (y + half) % 40.0
        if not (5.0 <= fx <= 35.0 and 5.0 <= fy <= 35.0):
            out.append((x, y, z))
    return np.asarray(out, dtype=np.float32)


def toy_workload() -> Workload:
    """Toy scene; iso V-pol tx at (0, 0, 10) m; 16 rx at 1.5 m; 1e5 rays,
    one reflection; 200x200 grid of 1 m cells at 1.5 m."""
    s = make_toy()
    rx = sample_street_points(s, 16, -95.0, 95.0, 1.5, seed=1)
    return Workload(s, [Device((0.0, 0.0, 10.0))], [Device(tuple(map(float, p))) for p in rx],
                    Grid(-100.0, -100.0, 1.0, 200, 200, 1.5), num_rays=100_000, max_depth=1)


def urban_tx(scene: Scene, pattern=PATTERN_ISO, pitch=0.0) -> Device:
    """2 m above the roof of building (3, 3), 0.5 m inside the roof corner that
    faces the central street crossing (a transmitter over the middle of a
    40 m roof would see almost nothing but its own roof)."""
    cx, cy, h, _ = scene.roofs[3 * 8 + 3]
    return Device((float(cx + 19.5), float(cy + 19.5), float(np.float32(h + 2.0))), yaw=0.0, pitch=pitch,
                  pattern=pattern)


def urban_workload(num_rays: int = 10_000_000) -> Workload:
    """Urban canyon: iso V-pol tx 2 m above a roof corner of building (3, 3);
    1e7 rays, three reflections; 400x400 grid of 1 m cells at 1.5 m; 16 rx."""
    s = make_urban(0)
    rx = sample_street_points(s, 16, -230.0, 230.0, 1.5, seed=1)
    return Workload(s, [urban_tx(s)], [Device(tuple(map(float, p))) for p in rx],
                    Grid(-200.0, -200.0, 1.0, 400, 400, 1.5), num_rays=num_rays, max_depth=3)


def diff_workload(num_rays: int = 1_000_000) -> Workload:
    """Differentiation case on the urban scene: TR 38.901 V-pol tx (yaw 0,
    pitch +10 deg) at the urban tx position, 256 street rx, 1e6 rays, depth 3."""
    s = make_urban(0)
    rx = sample_street_points(s, 256, -240.0, 240.0, 1.5, seed=2)
    return Workload(s, [urban_tx(s, PATTERN_TR38901, np.deg2rad(10.0))],
                    [Device(tuple(map(float, p))) for p in rx],
                    Grid(-200.0, -200.0, 1.0, 400, 400, 1.5), num_rays=num_rays, max_depth=3)


def city_workload(num_rays: int = 100_000_000, blocks: int = 50) -> Workload:
    """Large city: TR 38.901 V-pol tx (pitch +10 deg) 2 m above the tallest
    building within 150 m of the origin; 28 GHz, 1e8 rays, five reflections;
    2000x2000 grid of 1 m cells at 1.5 m; 4096 street rx."""
    s = make_city(0, blocks)
    best = None
    for (x, y, h, _) in s.roofs:
        if x * x + y * y <= 150.0 ** 2 and (best is None or h > best[2]):
            best = (x, y, h)
    tx = Device((float(best[0]), float(best[1]), float(np.float32(best[2] + 2.0))), 0.0,
                float(np.deg2rad(10.0)), 0.0, PATTERN_TR38901)
    half = 20.0 * blocks
    rx = _city_street_points(4096, half, 1.5, seed=1)
    return Workload(s, [tx], [Device(tuple(map(float, p))) for p in rx],
                    Grid(-half, -half, 1.0, int(2 * half), int(2 * half), 1.5),
                    num_rays=num_rays, max_depth=5)


def rooftop_tx_positions(scene: Scene, n: int, seed: int) -> np.ndarray:
    """n tx positions uniform over the rooftop area: building chosen with
    probability proportional to its footprint area, position uniform in its
    footprint bounding box, height roof + 2 m."""
    rng = np.random.default_rng(seed)
    areas = np.asarray([r[3] for r in scene.roofs], dtype=np.float64)
    idx = rng.choice(len(areas), size=n, p=areas / areas.sum())
    out = np.empty((n, 3), dtype=np.float32)
    for k, b in enumerate(idx):
        x0, x1, y0, y1 = scene.footprints[b]
        out[k] = (rng.uniform(x0, x1), rng.uniform(y0, y1), scene.roofs[b][2] + 2.0)
    return out


def random_rays(n: int, seed: int, lo=-60.0, hi=60.0, zlo=0.5, zhi=40.0):
    """Random ray origins in a box and isotropic unit directions (float32)."""
    rng = np.random.default_rng(seed)
    o = np.stack([rng.uniform(lo, hi, n), rng.uniform(lo, hi, n), rng.uniform(zlo, zhi, n)], 1)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)
