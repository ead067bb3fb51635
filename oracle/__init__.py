"""Plain double-precision CPU oracle of TV-superiorized proton-CT reconstruction.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
imports it and shares no code with it.

Thin ctypes wrapper over ``oracle.c`` (built with gcc -O2 -ffp-contract=off).
What each function computes, and the passage of arXiv 1803.01112 it follows,
is stated in ``oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle shared library (gcc, FP64, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=gnu11",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class OrGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("vx", C.c_double), ("vy", C.c_double), ("vz", C.c_double),
                ("ox", C.c_double), ("oy", C.c_double), ("oz", C.c_double)]


class OrMlpCfg(C.Structure):
    _fields_ = [("step_mm", C.c_double), ("log_term", C.c_int32), ("const_power", C.c_int32)]


_FP = C.POINTER(C.c_float)


class OrHist(C.Structure):
    _fields_ = [(n, _FP) for n in ("ex", "ey", "ez", "qx", "qy", "qz", "eth", "eps", "qth", "qps",
                                   "ux", "uy", "wepl")]


class OrParams(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("N", C.c_int32), ("alpha", C.c_double),
                ("tv_check", C.c_int32), ("variant", C.c_int32), ("tv_eps", C.c_double),
                ("seed", C.c_uint64), ("gamma", C.c_double), ("max_tries", C.c_int32)]


class OrState(C.Structure):
    _fields_ = [("k", C.c_int64), ("ell", C.c_int64), ("rng", C.c_uint64), ("seeded", C.c_int32)]


class OrStepLog(C.Structure):
    _fields_ = [("k", C.c_int32), ("n", C.c_int32), ("tries", C.c_int32), ("accepted", C.c_int32),
                ("ell_start", C.c_int64), ("phi_x", C.c_double), ("phi_z", C.c_double),
                ("gnorm", C.c_double), ("disagree", C.c_int32), ("pad", C.c_int32),
                ("worst_margin", C.c_double)]


class OrSystem(C.Structure):
    _fields_ = [("nh", C.c_int64), ("row_off", C.POINTER(C.c_int64)),
                ("idx", C.POINTER(C.c_int32)), ("chord", C.POINTER(C.c_double)),
                ("norm2", C.POINTER(C.c_double)), ("wepl", C.POINTER(C.c_double)),
                ("B", C.c_int64)]


HIST_FIELDS = ("ex", "ey", "ez", "qx", "qy", "qz", "eth", "eps", "qth", "qps", "ux", "uy", "wepl")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.or_mlp_sigmas.argtypes = [C.c_double, C.c_double, C.POINTER(OrMlpCfg), dp, dp]
        L.or_mlp_polyline.argtypes = [dp, C.POINTER(OrMlpCfg), dp, C.c_int64]
        L.or_mlp_polyline.restype = C.c_int64
        L.or_walk_polyline.argtypes = [C.POINTER(OrGrid), dp, C.c_int64, C.POINTER(C.c_int32), dp,
                                       C.c_int64, dp]
        L.or_walk_polyline.restype = C.c_int64
        L.or_build_rows.argtypes = [C.POINTER(OrGrid), C.POINTER(OrHist), C.c_int64,
                                    C.POINTER(OrMlpCfg), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int64), C.POINTER(C.c_int32), dp, dp]
        L.or_drop_sweep.argtypes = [C.c_int64, dp, C.c_int64, C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int32), dp, dp, dp, C.c_double, C.c_int64]
        L.or_tv.argtypes = [C.POINTER(OrGrid), dp, C.c_double]
        L.or_tv.restype = C.c_double
        L.or_tv_grad.argtypes = [C.POINTER(OrGrid), dp, C.c_double, dp]
        L.or_tv_grad.restype = C.c_double
        L.or_splitmix64_next.argtypes = [C.POINTER(C.c_uint64)]
        L.or_splitmix64_next.restype = C.c_uint64
        L.or_rand_ell.argtypes = [C.c_int64, C.c_int64, C.POINTER(C.c_uint64)]
        L.or_rand_ell.restype = C.c_int64
        L.or_superiorize.argtypes = [C.POINTER(OrGrid), C.POINTER(OrSystem), dp,
                                     C.POINTER(OrParams), C.c_int32, C.POINTER(OrState),
                                     C.POINTER(C.c_int64), C.POINTER(OrStepLog), C.c_int64,
                                     C.POINTER(C.c_int32), C.c_int64]
        L.or_superiorize.restype = C.c_int64
        ip = C.POINTER(C.c_int64)
        L.or_fbp_bin.argtypes = [C.POINTER(OrGrid), C.POINTER(OrHist), C.c_int64, C.c_int32,
                                 C.c_double, C.c_int32, dp, ip]
        L.or_fbp_filter.argtypes = [dp, C.c_int64, C.c_int32, C.c_double, dp]
        L.or_fbp_backproject.argtypes = [C.POINTER(OrGrid), dp, C.c_int32, C.c_double, C.c_int32,
                                         dp]
        L.or_median_slices.argtypes = [C.POINTER(OrGrid), dp, C.c_int32, dp]
        L.or_hull_counts.argtypes = [C.POINTER(OrGrid), C.POINTER(OrHist), C.c_int64, C.c_double,
                                     C.c_double, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.or_hull_counts.restype = None
        L.or_hull_decide.argtypes = [C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.c_int32, C.c_int32, C.POINTER(C.c_uint8)]
        L.or_hull_decide.restype = None
        L.or_log.argtypes = [C.c_double]
        L.or_log.restype = C.c_double
        L.or_set_threads.argtypes = [C.c_int32]
        L.or_set_threads.restype = None
        L.or_max_threads.argtypes = []
        L.or_max_threads.restype = C.c_int32
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _grid(g) -> OrGrid:
    return OrGrid(int(g.nx), int(g.ny), int(g.nz), float(g.vx), float(g.vy), float(g.vz),
                  float(g.ox), float(g.oy), float(g.oz))


def _cfg(step_mm, log_term=1, const_power=0) -> OrMlpCfg:
    return OrMlpCfg(float(step_mm), int(log_term), int(const_power))


# --------------------------------------------------------------------------- MLP
def mlp_sigmas(d1, L, log_term=1, const_power=0):
    """(Sigma1, Sigma2) as 2x2 arrays: scattering moments entry->d1 and d1->exit."""
    s1 = np.zeros(3)
    s2 = np.zeros(3)
    lib().or_mlp_sigmas(float(d1), float(L), C.byref(_cfg(1.0, log_term, const_power)), _dp(s1),
                        _dp(s2))
    return (np.array([[s1[0], s1[1]], [s1[1], s1[2]]]), np.array([[s2[0], s2[1]], [s2[1], s2[2]]]))


def mlp_polyline(h12, step_mm, log_term=1, const_power=0):
    """Polyline (entry, MLP vertices, exit) of one history as an (n, 3) array, or None
    when the history forms no row.  h12 = (ex,ey,ez,qx,qy,qz,eth,eps,qth,qps,ux,uy)."""
    h = np.ascontiguousarray(np.asarray(h12, dtype=np.float64))
    u = np.array([h[10], h[11]]) / np.hypot(h[10], h[11])
    L = (h[3] - h[0]) * u[0] + (h[4] - h[1]) * u[1]
    cap = int(np.ceil((abs(L) + 1.0) / step_mm)) + 4
    pts = np.zeros(3 * cap)
    n = lib().or_mlp_polyline(_dp(h), C.byref(_cfg(step_mm, log_term, const_power)), _dp(pts), cap)
    if n < 0:
        return None
    return pts[:3 * n].reshape(n, 3).copy()


def walk_polyline(grid, pts):
    """Row of one polyline: (int32 voxel indices, float64 chords in mm, ||a||^2)."""
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    g = _grid(grid)
    n2 = C.c_double(0.0)
    n = lib().or_walk_polyline(C.byref(g), _dp(pts), len(pts), None, None, 0, C.byref(n2))
    idx = np.zeros(max(n, 1), np.int32)
    ch = np.zeros(max(n, 1), np.float64)
    lib().or_walk_polyline(C.byref(g), _dp(pts), len(pts),
                           idx.ctypes.data_as(C.POINTER(C.c_int32)), _dp(ch), n, C.byref(n2))
    return idx[:n], ch[:n], n2.value


def _hist_struct(hist):
    arrs = {k: np.ascontiguousarray(hist[k], dtype=np.float32) for k in HIST_FIELDS}
    hs = OrHist(*[arrs[k].ctypes.data_as(_FP) for k in HIST_FIELDS])
    return hs, arrs


def build_rows(grid, hist, step_mm, log_term=1, const_power=0):
    """All rows of the system: dict(row_off int64[H+1], idx int32[nnz], chord f64[nnz],
    norm2 f64[H], wepl f64[H])."""
    hs, keep = _hist_struct(hist)
    nh = len(keep["ex"])
    g = _grid(grid)
    cfg = _cfg(step_mm, log_term, const_power)
    nnz = np.zeros(nh, np.int64)
    L = lib()
    L.or_build_rows(C.byref(g), C.byref(hs), nh, C.byref(cfg),
                    nnz.ctypes.data_as(C.POINTER(C.c_int64)), None, None, None, None)
    row_off = np.zeros(nh + 1, np.int64)
    np.cumsum(nnz, out=row_off[1:])
    tot = int(row_off[-1])
    idx = np.zeros(max(tot, 1), np.int32)
    chord = np.zeros(max(tot, 1), np.float64)
    norm2 = np.zeros(nh, np.float64)
    L.or_build_rows(C.byref(g), C.byref(hs), nh, C.byref(cfg),
                    nnz.ctypes.data_as(C.POINTER(C.c_int64)),
                    row_off.ctypes.data_as(C.POINTER(C.c_int64)),
                    idx.ctypes.data_as(C.POINTER(C.c_int32)), _dp(chord), _dp(norm2))
    return dict(row_off=row_off, idx=idx[:tot], chord=chord[:tot], norm2=norm2,
                wepl=keep["wepl"].astype(np.float64))


# --------------------------------------------------------------------------- DROP
def drop_sweep(x, rows, lam, B):
    """One DROP sweep over all blocks of B rows, in place on the float64 image x."""
    assert x.dtype == np.float64 and x.flags.c_contiguous
    lib().or_drop_sweep(x.size, _dp(x), len(rows["norm2"]),
                        rows["row_off"].ctypes.data_as(C.POINTER(C.c_int64)),
                        rows["idx"].ctypes.data_as(C.POINTER(C.c_int32)), _dp(rows["chord"]),
                        _dp(rows["norm2"]), _dp(rows["wepl"]), float(lam), int(B))
    return x


# --------------------------------------------------------------------------- TV
def tv(grid, x, eps=0.0):
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    return lib().or_tv(C.byref(_grid(grid)), _dp(x), float(eps))


def tv_grad(grid, x, eps=0.0):
    """(subgradient of TV as float64 array, ||g||^2)."""
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    g = np.zeros_like(x)
    n2 = lib().or_tv_grad(C.byref(_grid(grid)), _dp(x), float(eps), _dp(g))
    return g, n2


# --------------------------------------------------------------------------- schedule
def splitmix64(state: int, count: int):
    """(list of `count` SplitMix64 outputs, final state)."""
    s = C.c_uint64(state)
    out = [lib().or_splitmix64_next(C.byref(s)) for _ in range(count)]
    return out, s.value


def rand_ell(k: int, ell: int, state: int):
    s = C.c_uint64(state)
    r = lib().or_rand_ell(k, ell, C.byref(s))
    return r, s.value


def hull_counts(grid, hist, wepl_in, wepl_out):
    """Per voxel (x fastest): (in_count, out_count) -- histories whose straight
    entry-exit line crosses the voxel with WEPL >= wepl_in (space modelling)
    and with WEPL < wepl_out (space carving)."""
    hs, keep = _hist_struct(hist)
    n = len(keep["ex"])
    nvox = int(grid.nx) * int(grid.ny) * int(grid.nz)
    cin = np.zeros(nvox, np.int32)
    cout = np.zeros(nvox, np.int32)
    lib().or_hull_counts(C.byref(_grid(grid)), C.byref(hs), n, float(wepl_in), float(wepl_out),
                         cin.ctypes.data_as(C.POINTER(C.c_int32)),
                         cout.ctypes.data_as(C.POINTER(C.c_int32)))
    return cin, cout


def hull(grid, hist, wepl_in=1.0, wepl_out=1.0, min_in=1, max_out=0):
    """Hull mask (uint8 per voxel, x fastest): in_count >= min_in and
    out_count <= max_out."""
    cin, cout = hull_counts(grid, hist, wepl_in, wepl_out)
    out = np.zeros(len(cin), np.uint8)
    lib().or_hull_decide(len(cin), cin.ctypes.data_as(C.POINTER(C.c_int32)),
                         cout.ctypes.data_as(C.POINTER(C.c_int32)), int(min_in), int(max_out),
                         out.ctypes.data_as(C.POINTER(C.c_uint8)))
    return out


def log(x: float) -> float:
    """The oracle's natural logarithm (the MLP's Highland factor uses it)."""
    return float(lib().or_log(float(x)))


def set_threads(n: int) -> None:
    """Threads of the row formation (OpenMP); results do not depend on it."""
    lib().or_set_threads(int(n))


def max_threads() -> int:
    return int(lib().or_max_threads())


# --------------------------------------------------------------------------- driver
class Superiorizer:
    """K-cycle driver holding the oracle state (image, k, ell, RNG) between calls."""

    def __init__(self, grid, rows, x0, block_size):
        self.grid = grid
        self.g = _grid(grid)
        self.rows = rows
        self.x = np.ascontiguousarray(x0, dtype=np.float64).ravel().copy()
        self.sys = OrSystem(len(rows["norm2"]),
                            rows["row_off"].ctypes.data_as(C.POINTER(C.c_int64)),
                            rows["idx"].ctypes.data_as(C.POINTER(C.c_int32)),
                            _dp(rows["chord"]), _dp(rows["norm2"]), _dp(rows["wepl"]),
                            int(block_size))
        self.state = OrState(0, 0, 0, 0)
        self.ell_log = []
        self.steps = []

    def iterate(self, K, lam, N, alpha, tv_check=0, variant=0, tv_eps=0.0, seed=0, gamma=0.5,
                max_tries=100000, replay_tries=None):
        p = OrParams(float(lam), int(N), float(alpha), int(tv_check), int(variant), float(tv_eps),
                     int(seed), float(gamma), int(max_tries))
        nsteps = K * (1 if variant == 1 else N)
        cap = max(nsteps, 1)
        logs = (OrStepLog * cap)()
        ells = np.zeros(max(K, 1), np.int64)
        rp, rn = None, 0
        if replay_tries is not None:
            rt = np.ascontiguousarray(replay_tries, dtype=np.int32)
            self._rt = rt
            rp, rn = rt.ctypes.data_as(C.POINTER(C.c_int32)), len(rt)
        n = lib().or_superiorize(C.byref(self.g), C.byref(self.sys), _dp(self.x), C.byref(p),
                                 int(K), C.byref(self.state),
                                 ells.ctypes.data_as(C.POINTER(C.c_int64)), logs, cap, rp, rn)
        self.ell_log.extend(int(v) for v in ells[:K])
        recs = [dict(k=r.k, n=r.n, tries=r.tries, accepted=r.accepted, ell_start=r.ell_start,
                     phi_x=r.phi_x, phi_z=r.phi_z, gnorm=r.gnorm, disagree=r.disagree,
                     worst_margin=r.worst_margin) for r in logs[:min(n, cap)]]
        self.steps.extend(recs)
        return recs


# --------------------------------------------------------------------------- initial iterate
def fbp_lateral_bins(grid, tau):
    """Lateral bins covering the grid: 2 * ceil(R / tau) + 2, R the largest
    distance of a slice corner from the rotation axis."""
    xs = (float(grid.ox), float(grid.ox) + grid.nx * float(grid.vx))
    ys = (float(grid.oy), float(grid.oy) + grid.ny * float(grid.vy))
    R = max(np.hypot(x, y) for x in xs for y in ys)
    return 2 * int(np.ceil(R / tau)) + 2


def fbp_bin(grid, hist, A, tau, nt):
    """Mean WEPL per (angle, slice, lateral) bin, and the bins' history counts."""
    hs, keep = _hist_struct(hist)
    nh = len(keep["ex"])
    p = np.zeros(A * grid.nz * nt, np.float64)
    cnt = np.zeros(A * grid.nz * nt, np.int64)
    lib().or_fbp_bin(C.byref(_grid(grid)), C.byref(hs), nh, int(A), float(tau), int(nt), _dp(p),
                     cnt.ctypes.data_as(C.POINTER(C.c_int64)))
    return p, cnt


def fbp_filter(p, nt, tau):
    p = np.ascontiguousarray(p, dtype=np.float64)
    q = np.zeros_like(p)
    lib().or_fbp_filter(_dp(p), p.size // nt, int(nt), float(tau), _dp(q))
    return q


def fbp_backproject(grid, q, A, tau, nt):
    q = np.ascontiguousarray(q, dtype=np.float64)
    x = np.zeros(grid.nvox, np.float64)
    lib().or_fbp_backproject(C.byref(_grid(grid)), _dp(q), int(A), float(tau), int(nt), _dp(x))
    return x


def median_slices(grid, x, r):
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    y = np.zeros_like(x)
    lib().or_median_slices(C.byref(_grid(grid)), _dp(x), int(r), _dp(y))
    return y


def fbp_initial(grid, hist, A, tau=None, median_r=2, clip=True):
    """Initial iterate: FBP of the binned histories, negatives set to 0
    (clip), then the in-slice median of radius median_r (0: none)."""
    tau = float(grid.vx) if tau is None else float(tau)
    nt = fbp_lateral_bins(grid, tau)
    p, _ = fbp_bin(grid, hist, A, tau, nt)
    x = fbp_backproject(grid, fbp_filter(p, nt, tau), A, tau, nt)
    if clip:
        x = np.maximum(x, 0.0)
    if median_r > 0:
        x = median_slices(grid, x, median_r)
    return x
