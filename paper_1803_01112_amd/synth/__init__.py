"""Seeded synthetic inputs: voxel grids, a cylinder phantom with six material
inserts, proton histories through it, and the hull-masked initial image.

This module is an input generator only and holds none of the
reconstruction's arithmetic.  It stands in for the paper's Catphan CTP404
data (arXiv 1803.01112, Section III-C), taking its geometry: a 15 cm
cylinder of RSP 1.0 with 12.2 mm inserts on a 120 mm ring, 90 projection
angles of 4 degrees, 200 MeV protons, WEPL with 1 % Gaussian noise.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import NamedTuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None

HIST_FIELDS = ("ex", "ey", "ez", "qx", "qy", "qz", "eth", "eps", "qth", "qps", "ux", "uy", "wepl")
INSERT_RSP = (0.0012, 0.6, 0.95, 1.05, 1.3, 1.7)


class Grid(NamedTuple):
    """nx*ny*nz voxels of vx*vy*vz mm; (ox, oy, oz) is the corner of voxel 0; x fastest."""
    nx: int
    ny: int
    nz: int
    vx: float
    vy: float
    vz: float
    ox: float
    oy: float
    oz: float

    @property
    def nvox(self) -> int:
        return self.nx * self.ny * self.nz


def centered_grid(nx, ny, nz, vx, vy, vz) -> Grid:
    """Grid centred on the origin (the phantom axis is z through the origin)."""
    return Grid(nx, ny, nz, float(vx), float(vy), float(vz),
                -0.5 * nx * vx, -0.5 * ny * vy, -0.5 * nz * vz)


@dataclass
class Phantom:
    radius: float
    zlo: float
    zhi: float
    inserts: list = field(default_factory=list)   # (cx, cy, r, rsp)
    rsp_bg: float = 1.0

    def rsp_at(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        out = np.where(x * x + y * y <= self.radius ** 2, self.rsp_bg, 0.0)
        for cx, cy, r, rsp in self.inserts:
            inside = (x - cx) ** 2 + (y - cy) ** 2 <= r * r
            out = np.where(inside & (x * x + y * y <= self.radius ** 2), rsp, out)
        return out


def catphan_like(grid: Grid, diameter: float) -> Phantom:
    """Cylinder of the given diameter; six inserts of diameter 0.0813 D on a ring of
    radius 0.4 D at 0, 60, ..., 300 degrees with RSP 0.0012 ... 1.7."""
    ins = []
    for q, rsp in enumerate(INSERT_RSP):
        a = math.radians(60.0 * q)
        ins.append((0.4 * diameter * math.cos(a), 0.4 * diameter * math.sin(a),
                    0.5 * 0.0813 * diameter, rsp))
    return Phantom(0.5 * diameter, grid.oz, grid.oz + grid.nz * grid.vz, ins)


def voxel_centres(grid: Grid):
    x = grid.ox + (np.arange(grid.nx) + 0.5) * grid.vx
    y = grid.oy + (np.arange(grid.ny) + 0.5) * grid.vy
    return np.meshgrid(x, y, indexing="xy")


def initial_image(grid: Grid, phantom: Phantom) -> np.ndarray:
    """1.0 for voxels whose centre lies inside the phantom cylinder, else 0 (float32)."""
    X, Y = voxel_centres(grid)
    sl = (X * X + Y * Y <= phantom.radius ** 2).astype(np.float32)
    return np.ascontiguousarray(np.broadcast_to(sl, (grid.nz, grid.ny, grid.nx))).ravel().copy()


def truth_image(grid: Grid, phantom: Phantom) -> np.ndarray:
    X, Y = voxel_centres(grid)
    sl = phantom.rsp_at(X, Y).astype(np.float32)
    return np.ascontiguousarray(np.broadcast_to(sl, (grid.nz, grid.ny, grid.nx))).ravel().copy()


# --------------------------------------------------------------------------- C generator
class _Phantom(C.Structure):
    _fields_ = [("R", C.c_double), ("n_ins", C.c_int32),
                ("ins_x", C.c_double * 8), ("ins_y", C.c_double * 8), ("ins_r", C.c_double * 8),
                ("ins_rsp", C.c_double * 8), ("rsp_bg", C.c_double),
                ("zlo", C.c_double), ("zhi", C.c_double)]


class _Cfg(C.Structure):
    _fields_ = [("n_hist", C.c_int64), ("n_angles", C.c_int32), ("two_d", C.c_int32),
                ("e0_mev", C.c_double), ("step_mm", C.c_double), ("lat_frac", C.c_double),
                ("v_margin_mm", C.c_double), ("noise_frac", C.c_double), ("seed", C.c_uint64),
                ("first", C.c_int64), ("count", C.c_int64)]


_FP = C.POINTER(C.c_float)


class _Out(C.Structure):
    _fields_ = [(n, _FP) for n in HIST_FIELDS]


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-std=gnu11", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = C.CDLL(_LIB)
        _lib.sy_generate.argtypes = [C.POINTER(_Phantom), C.POINTER(_Cfg), C.POINTER(_Out)]
        _lib.sy_generate.restype = C.c_int64
    return _lib


def generate(grid: Grid, phantom: Phantom, n_hist: int, n_angles: int, seed: int, *,
             two_d: bool = False, first: int = 0, count: int | None = None,
             step_mm: float = 0.5, e0_mev: float = 200.0, noise_frac: float = 0.01,
             lat_frac: float = 0.95, v_margin_mm: float = 0.5) -> dict:
    """Histories [first, first+count) of an n_hist-history scan: dict of 13 float32 arrays
    (entry/exit positions in mm, entry/exit slopes dt/du and dv/du, beam axis (ux, uy),
    WEPL in mm).  Angle-major order; lateral position uniform within each angle."""
    if count is None:
        count = n_hist - first
    p = _Phantom()
    p.R = phantom.radius
    p.n_ins = len(phantom.inserts)
    for q, (cx, cy, r, rsp) in enumerate(phantom.inserts):
        p.ins_x[q], p.ins_y[q], p.ins_r[q], p.ins_rsp[q] = cx, cy, r, rsp
    p.rsp_bg = phantom.rsp_bg
    p.zlo, p.zhi = phantom.zlo, phantom.zhi
    cfg = _Cfg(int(n_hist), int(n_angles), int(bool(two_d)), float(e0_mev), float(step_mm),
               float(lat_frac), float(v_margin_mm), float(noise_frac), int(seed) & (2**64 - 1),
               int(first), int(count))
    out = {k: np.zeros(count, np.float32) for k in HIST_FIELDS}
    o = _Out(*[out[k].ctypes.data_as(_FP) for k in HIST_FIELDS])
    _load().sy_generate(C.byref(p), C.byref(cfg), C.byref(o))
    return out


def line_histories(p0, p1, wepl) -> dict:
    """Histories from explicit straight entry / exit points (mm) and WEPL:
    zero slopes, the beam axis along each line's in-plane direction."""
    p0 = np.asarray(p0, np.float64)
    p1 = np.asarray(p1, np.float64)
    d = p1[:, :2] - p0[:, :2]
    u = d / np.linalg.norm(d, axis=1, keepdims=True)
    z = np.zeros(len(p0))
    h = dict(ex=p0[:, 0], ey=p0[:, 1], ez=p0[:, 2], qx=p1[:, 0], qy=p1[:, 1], qz=p1[:, 2],
             eth=z, eps=z, qth=z, qps=z, ux=u[:, 0], uy=u[:, 1], wepl=np.asarray(wepl, np.float64))
    return {k: np.ascontiguousarray(v, np.float32) for k in HIST_FIELDS for v in [h[k]]}


def miss_histories(grid: Grid, radius: float, n: int, seed: int, noise_mm: float = 0.3) -> dict:
    """Protons that pass beside a cylinder of the given radius (axis z
    through the origin): straight lines across the grid's slab at uniform
    angles with lateral offsets between radius + 0.5 mm and the grid's
    corner, their WEPL only the detector noise N(0, noise_mm)."""
    rng = np.random.default_rng(seed)
    half = 0.5 * math.hypot(grid.nx * grid.vx, grid.ny * grid.vy)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    t = rng.uniform(radius + 0.5, max(half, radius + 1.0), n) * rng.choice([-1.0, 1.0], n)
    v = rng.uniform(grid.oz, grid.oz + grid.nz * grid.vz, n)
    u = np.stack([np.cos(phi), np.sin(phi)], 1)
    c = t[:, None] * np.stack([-np.sin(phi), np.cos(phi)], 1)
    p0 = np.concatenate([c - (half + 5.0) * u, v[:, None]], 1)
    p1 = np.concatenate([c + (half + 5.0) * u, v[:, None]], 1)
    return line_histories(p0, p1, rng.normal(0.0, noise_mm, n))


# --------------------------------------------------------------------------- workloads
@dataclass
class Workload:
    """A named synthetic reconstruction problem shaped like the paper's scans."""
    name: str
    grid: Grid
    diameter: float
    n_hist: int
    n_angles: int
    seed: int
    two_d: bool = False

    @property
    def phantom(self) -> Phantom:
        return catphan_like(self.grid, self.diameter)

    def histories(self, first: int = 0, count: int | None = None, **kw) -> dict:
        return generate(self.grid, self.phantom, self.n_hist, self.n_angles, self.seed,
                        two_d=self.two_d, first=first, count=count, **kw)

    def initial_image(self) -> np.ndarray:
        return initial_image(self.grid, self.phantom)


def workload(name: str, n_hist: int | None = None) -> Workload:
    """Named workloads:
    slice64   -- 64x64 voxels of 2 mm (one slice), 96 mm cylinder, 60k histories at 90 angles
    vol200    -- 200x200x16 voxels of 1x1x2.5 mm, 150 mm cylinder, 20M histories at 180 angles
    vol256    -- 256x256x32 voxels of 1x1x2.5 mm, 192 mm cylinder, 60M histories at 360 angles
    slab256   -- 256x256x2 voxels of 1x1x2.5 mm (two slices of vol256), 3.75M histories
    vol64     -- 64x64x4 voxels of 1x1x2.5 mm (smallest serving grid), 48 mm cylinder
    vol128    -- 128x128x8 voxels of 1x1x2.5 mm, 96 mm cylinder
    n_hist overrides the history count (a smaller scan over the same angles)."""
    base = 1803011120
    table = {
        "slice64": (centered_grid(64, 64, 1, 2.0, 2.0, 2.0), 96.0, 60_000, 90, base + 0, True),
        "vol200": (centered_grid(200, 200, 16, 1.0, 1.0, 2.5), 150.0, 20_000_000, 180, base + 1,
                   False),
        "vol256": (centered_grid(256, 256, 32, 1.0, 1.0, 2.5), 192.0, 60_000_000, 360, base + 3,
                   False),
        "slab256": (centered_grid(256, 256, 2, 1.0, 1.0, 2.5), 192.0, 3_750_000, 360, base + 3,
                    False),
        "vol64": (centered_grid(64, 64, 4, 1.0, 1.0, 2.5), 48.0, 1_000_000, 90, base + 4, False),
        "vol128": (centered_grid(128, 128, 8, 1.0, 1.0, 2.5), 96.0, 4_000_000, 180, base + 4,
                   False),
    }
    g, d, nh, na, seed, two_d = table[name]
    return Workload(name, g, d, int(n_hist if n_hist is not None else nh), na, seed, two_d)
