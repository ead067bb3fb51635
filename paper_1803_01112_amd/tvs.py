"""Python binding of libtvs (include/tvs.h): argument marshalling only.

Every step of the reconstruction runs in the gfx950 kernels behind the C
ABI; this module converts arguments (numpy arrays for host memory, torch
CUDA tensors for device memory, torch streams or raw hipStream_t handles)
and raises TvsError on a failing status.  There is no fallback: if the
shared library is missing the import of the library fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from ._build import LIB

HIST_FIELDS = ("ex", "ey", "ez", "qx", "qy", "qz", "eth", "eps", "qth", "qps", "ux", "uy", "wepl")

TVS_OK, TVS_EINVAL, TVS_ENOMEM, TVS_EDEVICE, TVS_ESTATE, TVS_ERANGE = 0, -1, -2, -3, -4, -5
PATH_MODES = {"otf": 0, "f32": 1, "f16": 2, "q16": 3}
VARIANTS = {"ntvs": 0, "otvs": 1, "decoupled": 2}

EXPORTED = ("tvs_config_default", "tvs_create", "tvs_destroy", "tvs_load_histories",
            "tvs_set_image", "tvs_iterate", "tvs_get_image", "tvs_get_stats", "tvs_get_step_log",
            "tvs_debug_rows", "tvs_strerror", "tvs_last_error", "tvs_iterate_batch",
            "tvs_get_batch_image", "tvs_server_config_default", "tvs_server_create",
            "tvs_server_footprint", "tvs_server_submit", "tvs_server_query", "tvs_server_wait",
            "tvs_server_get_counters", "tvs_server_destroy", "tvs_autotune", "tvs_initial_fbp",
            "tvs_initial_fbp_noalloc", "tvs_hull_detect",
            "tvs_autotune_batch")


class TvsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("vx", C.c_double), ("vy", C.c_double), ("vz", C.c_double),
                ("ox", C.c_double), ("oy", C.c_double), ("oz", C.c_double)]


class Config(C.Structure):
    _fields_ = [("block_size", C.c_int32), ("path_mode", C.c_int32), ("mlp_step_mm", C.c_double),
                ("mlp_log_term", C.c_int32), ("mlp_const_power", C.c_int32),
                ("chunk_histories", C.c_int64), ("hbm_budget_bytes", C.c_uint64),
                ("device", C.c_int32), ("max_tries", C.c_int32), ("sweep_kernel", C.c_int32),
                ("tile_threads", C.c_int32), ("time_sample", C.c_int32),
                ("fill_wgs_per_cu", C.c_int32), ("fill_wide_pct", C.c_int32)]


_FP = C.POINTER(C.c_float)


class Histories(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in HIST_FIELDS]


class Params(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("N", C.c_int32), ("alpha", C.c_double),
                ("tv_check", C.c_int32), ("variant", C.c_int32), ("tv_eps", C.c_double),
                ("seed", C.c_uint64), ("gamma", C.c_double)]


class FbpParams(C.Structure):
    _fields_ = [("n_angles", C.c_int32), ("median_radius", C.c_int32), ("t_bin_mm", C.c_double),
                ("clip_negative", C.c_int32), ("pad", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("k", C.c_int64), ("ell", C.c_int64), ("n_hist", C.c_int64),
                ("n_skipped", C.c_int64), ("nnz", C.c_int64), ("steps", C.c_int64),
                ("tries", C.c_int64), ("max_row_nnz", C.c_int64), ("last_sweep_ms", C.c_double),
                ("last_tv_ms", C.c_double), ("last_rows_ms", C.c_double),
                ("device_bytes", C.c_uint64), ("tv_ms_total", C.c_double),
                ("sweep_ms_total", C.c_double), ("rows_ms_total", C.c_double),
                ("drop_ms_total", C.c_double), ("cycles_timed", C.c_int64),
                ("rows_launches", C.c_int64), ("drop_launches", C.c_int64),
                ("k1_ms_total", C.c_double), ("k2_ms_total", C.c_double),
                ("k_samples", C.c_int64), ("batch_ms_total", C.c_double), ("batch_cycles", C.c_int64),
                ("batch_size", C.c_int32), ("pad", C.c_int32)]


class BatchTuneResult(C.Structure):
    _fields_ = [("threads", C.c_int32), ("group", C.c_int32), ("ms_per_block", C.c_double),
                ("from_cache", C.c_int32), ("n_candidates", C.c_int32),
                ("cand_threads", C.c_int32 * 8), ("cand_group", C.c_int32 * 8),
                ("cand_ms", C.c_double * 8)]


class HullParams(C.Structure):
    _fields_ = [("wepl_in_mm", C.c_double), ("wepl_out_mm", C.c_double), ("min_in", C.c_int32),
                ("max_out", C.c_int32), ("mask_image", C.c_int32), ("pad", C.c_int32)]


class StepLog(C.Structure):
    _fields_ = [("k", C.c_int32), ("n", C.c_int32), ("tries", C.c_int32), ("accepted", C.c_int32),
                ("ell_start", C.c_int64), ("phi_x", C.c_double), ("phi_z", C.c_double),
                ("gnorm", C.c_double)]


class TuneResult(C.Structure):
    _fields_ = [("tile_threads", C.c_int32), ("sweep_kernel", C.c_int32),
                ("ms_per_block", C.c_double), ("from_cache", C.c_int32),
                ("n_candidates", C.c_int32), ("cand_threads", C.c_int32 * 8),
                ("cand_sweep", C.c_int32 * 8), ("cand_ms", C.c_double * 8),
                ("fill_wide_pct", C.c_int32), ("n_fill", C.c_int32), ("cand_pct", C.c_int32 * 8),
                ("cand_sweep_ms", C.c_double * 8)]


class ServerConfig(C.Structure):
    _fields_ = [("device", C.c_int32), ("max_active", C.c_int32),
                ("hbm_budget_bytes", C.c_uint64), ("chunk_histories", C.c_int64),
                ("simulate", C.c_int32), ("pad", C.c_int32),
                ("sim_ns_per_history_cycle", C.c_double)]


class Request(C.Structure):
    _fields_ = [("grid", Grid), ("block_size", C.c_int32), ("path_mode", C.c_int32),
                ("params", Params), ("K", C.c_int32), ("pad", C.c_int32), ("n", C.c_int64),
                ("h", Histories), ("x0", C.c_void_p)]


class RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("submit_ms", C.c_double),
                ("admit_ms", C.c_double), ("done_ms", C.c_double), ("bytes", C.c_uint64),
                ("admit_order", C.c_int64)]


class ServerCounters(C.Structure):
    _fields_ = [("budget_bytes", C.c_uint64), ("in_use_bytes", C.c_uint64),
                ("peak_bytes", C.c_uint64), ("active", C.c_int32), ("peak_active", C.c_int32),
                ("queued", C.c_int32), ("pad", C.c_int32), ("completed", C.c_int64),
                ("failed", C.c_int64)]


_lib = None


def load_library(path: str = LIB):
    """Loads libtvs.so (built by __graft_entry__.build); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libtvs.so not built at {path}: run __graft_entry__.build() first")
    # PyTorch's wheel carries its own HIP and HSA runtimes, which its
    # libraries request under other file names than the system's.  Loaded
    # first, they also serve libtvs (same sonames), so the process holds one
    # runtime; loaded after libtvs, they would be a second runtime, and
    # PyTorch would then find no GPU.
    import torch  # noqa: F401
    L = C.CDLL(path)
    P = C.POINTER
    L.tvs_config_default.argtypes = [P(Config)]
    L.tvs_config_default.restype = None
    L.tvs_create.argtypes = [P(Grid), P(Config), P(C.c_void_p)]
    L.tvs_destroy.argtypes = [C.c_void_p]
    L.tvs_destroy.restype = None
    L.tvs_load_histories.argtypes = [C.c_void_p, C.c_int64, P(Histories), C.c_int, C.c_void_p]
    L.tvs_set_image.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
    L.tvs_iterate.argtypes = [C.c_void_p, P(Params), C.c_int32, C.c_void_p]
    L.tvs_get_image.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
    L.tvs_get_stats.argtypes = [C.c_void_p, P(Stats)]
    L.tvs_iterate_batch.argtypes = [C.c_void_p, P(Params), C.c_int32, C.c_int32, C.c_void_p]
    L.tvs_get_batch_image.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int, C.c_void_p]
    L.tvs_initial_fbp.argtypes = [C.c_void_p, P(FbpParams), C.c_void_p, C.c_int, C.c_void_p]
    L.tvs_initial_fbp_noalloc.argtypes = [C.c_void_p, P(FbpParams), C.c_void_p, C.c_int,
                                          C.c_void_p]
    L.tvs_get_step_log.argtypes = [C.c_void_p, P(StepLog), C.c_int64, P(C.c_int64)]
    L.tvs_hull_detect.argtypes = [C.c_void_p, P(HullParams), C.c_void_p, C.c_int, C.c_void_p]
    L.tvs_hull_detect.restype = C.c_int
    L.tvs_debug_rows.argtypes = [C.c_void_p, C.c_int64, C.c_int64, P(C.c_int64), P(C.c_int32),
                                 _FP, _FP, C.c_int64]
    L.tvs_strerror.argtypes = [C.c_int]
    L.tvs_strerror.restype = C.c_char_p
    L.tvs_last_error.argtypes = [C.c_void_p]
    L.tvs_last_error.restype = C.c_char_p
    L.tvs_autotune.argtypes = [C.c_void_p, C.c_double, C.c_char_p, P(TuneResult), C.c_void_p]
    L.tvs_autotune.restype = C.c_int
    L.tvs_autotune_batch.argtypes = [C.c_void_p, P(Params), C.c_int32, C.c_char_p,
                                     P(BatchTuneResult), C.c_void_p]
    L.tvs_autotune_batch.restype = C.c_int
    L.tvs_server_config_default.argtypes = [P(ServerConfig)]
    L.tvs_server_config_default.restype = None
    L.tvs_server_create.argtypes = [P(ServerConfig), P(C.c_void_p)]
    L.tvs_server_footprint.argtypes = [C.c_void_p, P(Request)]
    L.tvs_server_footprint.restype = C.c_uint64
    L.tvs_server_submit.argtypes = [C.c_void_p, P(Request), P(C.c_int64)]
    L.tvs_server_query.argtypes = [C.c_void_p, C.c_int64, P(RequestInfo)]
    L.tvs_server_wait.argtypes = [C.c_void_p, C.c_int64, _FP, C.c_int64, P(RequestInfo)]
    L.tvs_server_get_counters.argtypes = [C.c_void_p, P(ServerCounters)]
    L.tvs_server_destroy.argtypes = [C.c_void_p]
    L.tvs_server_destroy.restype = None
    for name in ("tvs_server_create", "tvs_server_submit", "tvs_server_query", "tvs_server_wait",
                 "tvs_server_get_counters"):
        getattr(L, name).restype = C.c_int
    for name in ("tvs_create", "tvs_load_histories", "tvs_set_image", "tvs_iterate",
                 "tvs_get_image", "tvs_get_stats", "tvs_get_step_log", "tvs_debug_rows",
                 "tvs_iterate_batch", "tvs_get_batch_image", "tvs_initial_fbp",
                 "tvs_initial_fbp_noalloc"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(int(stream.cuda_stream))


def _is_device(a) -> bool:
    return hasattr(a, "is_cuda") and bool(a.is_cuda)


def _ptr(a):
    """(pointer, on_device, keep-alive) of a float32 array or tensor."""
    if _is_device(a):
        import torch
        if a.dtype != torch.float32 or not a.is_contiguous():
            raise TypeError("device arrays must be contiguous float32 tensors")
        return C.c_void_p(a.data_ptr()), 1, a
    arr = np.ascontiguousarray(np.asarray(a), dtype=np.float32)
    return C.c_void_p(arr.ctypes.data), 0, arr


def _out_ptr(out, n, stream):
    """(pointer, on_device, stream handle, wait) of an output buffer of at
    least n float32 values.  A device tensor must be contiguous float32;
    without an explicit stream its copy is queued on torch's current stream
    when that is a stream of its own, so later torch work there sees it.
    torch's default stream has the null handle, which the library reads as
    the context's own stream: then `wait` is set and the caller synchronises
    the device after the call.  A host array must be a writeable,
    C-contiguous float32 array."""
    if _is_device(out):
        import torch
        if out.dtype != torch.float32 or not out.is_contiguous():
            raise TypeError("device outputs must be contiguous float32 tensors")
        if out.numel() < n:
            raise ValueError(f"output holds {out.numel()} values, {n} needed")
        if stream is None:
            cur = torch.cuda.current_stream(out.device)
            if int(cur.cuda_stream) != 0:
                return C.c_void_p(out.data_ptr()), 1, _stream_handle(cur), False
            return C.c_void_p(out.data_ptr()), 1, None, True
        return C.c_void_p(out.data_ptr()), 1, _stream_handle(stream), False
    if not isinstance(out, np.ndarray) or out.dtype != np.float32 or \
            not out.flags["C_CONTIGUOUS"] or not out.flags["WRITEABLE"]:
        raise TypeError("host outputs must be writeable C-contiguous float32 arrays")
    if out.size < n:
        raise ValueError(f"output holds {out.size} values, {n} needed")
    return C.c_void_p(out.ctypes.data), 0, _stream_handle(stream), False


def _settle(out, wait):
    """After a call that wrote device tensor `out` on the context's own
    stream: wait for the device, so that later torch work reads the result."""
    if wait:
        import torch
        torch.cuda.synchronize(out.device)


def _inputs_ready(arrays, stream):
    """Device inputs produced on torch's current stream are complete before
    the library (on its own stream when none is given) reads them."""
    if stream is None:
        for a in arrays:
            if _is_device(a):
                import torch
                torch.cuda.current_stream(a.device).synchronize()
                return


def grid_struct(g) -> Grid:
    return Grid(int(g.nx), int(g.ny), int(g.nz), float(g.vx), float(g.vy), float(g.vz),
                float(g.ox), float(g.oy), float(g.oz))


def default_config() -> Config:
    cfg = Config()
    load_library().tvs_config_default(C.byref(cfg))
    return cfg


class Context:
    """One reconstruction context (tvs_ctx): grid, histories, image and cycle state."""

    def __init__(self, grid, *, block_size=3200, path_mode="otf", mlp_step_mm=0.0,
                 mlp_log_term=True, mlp_const_power=False, chunk_histories=0,
                 hbm_budget_bytes=0, device=0, max_tries=0, sweep_kernel=0, tile_threads=0,
                 time_sample=0, fill_wgs_per_cu=0, fill_wide_pct=-1):
        self._L = load_library()
        self.grid = grid
        self.nvox = int(grid.nx) * int(grid.ny) * int(grid.nz)
        cfg = default_config()
        cfg.block_size = int(block_size)
        cfg.path_mode = PATH_MODES[path_mode] if isinstance(path_mode, str) else int(path_mode)
        cfg.mlp_step_mm = float(mlp_step_mm)
        cfg.mlp_log_term = int(bool(mlp_log_term))
        cfg.mlp_const_power = int(bool(mlp_const_power))
        cfg.chunk_histories = int(chunk_histories)
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.device = int(device)
        cfg.max_tries = int(max_tries)
        cfg.sweep_kernel = int(sweep_kernel)
        cfg.tile_threads = int(tile_threads)
        cfg.time_sample = int(time_sample)
        cfg.fill_wgs_per_cu = int(fill_wgs_per_cu)
        cfg.fill_wide_pct = int(fill_wide_pct)
        self.cfg = cfg
        h = C.c_void_p()
        g = grid_struct(grid)
        rc = self._L.tvs_create(C.byref(g), C.byref(cfg), C.byref(h))
        if rc != TVS_OK:
            raise TvsError(rc, "tvs_create: " + self._L.tvs_strerror(rc).decode())
        self._h = h

    # ------------------------------------------------------------------ helpers
    def _check(self, rc, what):
        if rc != TVS_OK:
            msg = self._L.tvs_last_error(self._h).decode() or self._L.tvs_strerror(rc).decode()
            raise TvsError(rc, f"{what}: {msg}")

    def close(self):
        if getattr(self, "_h", None):
            self._L.tvs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------------ calls
    def load_histories(self, hist: dict, stream=None):
        n = len(hist["ex"])
        ptrs, keep, dev = {}, [], None
        for k in HIST_FIELDS:
            p, d, ka = _ptr(hist[k])
            if len(ka) != n:
                raise ValueError("history streams differ in length")
            if dev is None:
                dev = d
            elif dev != d:
                raise ValueError("mix of host and device history streams")
            ptrs[k] = p
            keep.append(ka)
        hs = Histories(*[ptrs[k] for k in HIST_FIELDS])
        _inputs_ready(keep, stream)
        rc = self._L.tvs_load_histories(self._h, n, C.byref(hs), int(dev or 0),
                                        _stream_handle(stream))
        self._check(rc, "tvs_load_histories")

    def set_image(self, x, stream=None):
        p, d, keep = _ptr(x)
        if len(keep.reshape(-1)) != self.nvox:
            raise ValueError("image size does not match the grid")
        _inputs_ready([keep], stream)
        self._check(self._L.tvs_set_image(self._h, p, d, _stream_handle(stream)), "tvs_set_image")

    def iterate(self, K, lam, N, alpha, tv_check=False, variant="ntvs", tv_eps=0.0, seed=0,
                gamma=0.5, stream=None):
        v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        p = Params(float(lam), int(N), float(alpha), int(bool(tv_check)), v, float(tv_eps),
                   int(seed) & (2**64 - 1), float(gamma))
        self._check(self._L.tvs_iterate(self._h, C.byref(p), int(K), _stream_handle(stream)),
                    "tvs_iterate")

    @staticmethod
    def _settings(settings):
        S = len(settings)
        arr = (Params * max(S, 1))()
        for q, st in enumerate(settings):
            v = st.get("variant", "ntvs")
            v = VARIANTS[v] if isinstance(v, str) else int(v)
            arr[q] = Params(float(st["lam"]), int(st["N"]), float(st["alpha"]),
                            int(bool(st.get("tv_check", False))), v, float(st.get("tv_eps", 0.0)),
                            int(st.get("seed", 0)) & (2**64 - 1), float(st.get("gamma", 0.5)))
        return S, arr

    def iterate_batch(self, K, settings, stream=None):
        """K cycles of S settings together; settings: list of dicts with keys
        lam, N, alpha and optionally variant, tv_eps, seed, gamma."""
        S, arr = self._settings(settings)
        self._check(self._L.tvs_iterate_batch(self._h, arr, S, int(K), _stream_handle(stream)),
                    "tvs_iterate_batch")

    def autotune_batch(self, settings, cache_path=None, stream=None):
        """Times the batched step's shapes (threads x settings per LDS pass)
        for these settings and keeps the fastest; returns a dict."""
        S, arr = self._settings(settings)
        r = BatchTuneResult()
        cp = cache_path.encode() if cache_path else None
        self._check(self._L.tvs_autotune_batch(self._h, arr, S, cp, C.byref(r),
                                               _stream_handle(stream)), "tvs_autotune_batch")
        return dict(threads=r.threads, group=r.group, ms_per_block=r.ms_per_block,
                    from_cache=bool(r.from_cache),
                    candidates=[dict(threads=r.cand_threads[q], group=r.cand_group[q],
                                     ms=r.cand_ms[q]) for q in range(r.n_candidates)])

    def autotune(self, lam=1e-4, cache_path=None, stream=None):
        """Times the launch-shape candidates and keeps the fastest; returns a dict."""
        r = TuneResult()
        cp = cache_path.encode() if cache_path else None
        self._check(self._L.tvs_autotune(self._h, float(lam), cp, C.byref(r),
                                         _stream_handle(stream)), "tvs_autotune")
        n = r.n_candidates
        return dict(tile_threads=r.tile_threads, sweep_kernel=r.sweep_kernel,
                    ms_per_block=r.ms_per_block, from_cache=bool(r.from_cache),
                    candidates=[dict(threads=r.cand_threads[q], sweep=r.cand_sweep[q],
                                     ms=r.cand_ms[q]) for q in range(n)],
                    fill_wide_pct=r.fill_wide_pct,
                    fill_candidates=[dict(pct=r.cand_pct[q], ms=r.cand_sweep_ms[q])
                                     for q in range(r.n_fill)])

    def get_batch_image(self, s, out=None, stream=None):
        if out is None:
            out = np.zeros(self.nvox, np.float32)
        p, d, st, wait = _out_ptr(out, self.nvox, stream)
        self._check(self._L.tvs_get_batch_image(self._h, int(s), p, d, st), "tvs_get_batch_image")
        _settle(out, wait)
        return out

    def get_image(self, out=None, stream=None):
        if out is None:
            out = np.zeros(self.nvox, np.float32)
        p, d, st, wait = _out_ptr(out, self.nvox, stream)
        self._check(self._L.tvs_get_image(self._h, p, d, st), "tvs_get_image")
        _settle(out, wait)
        return out

    def initial_fbp(self, n_angles, median_radius=2, t_bin_mm=0.0, clip_negative=True, out=None,
                    stream=None):
        """Initial iterate by filtered backprojection of the loaded histories and
        an in-slice median (tvs_initial_fbp); it becomes the context image.
        Returns it (float32, x fastest) in `out` (host array or device tensor)
        or a new host array."""
        prm = FbpParams(int(n_angles), int(median_radius), float(t_bin_mm), int(bool(clip_negative)), 0)
        if out is None:
            out = np.zeros(self.nvox, np.float32)
        p, d, st, wait = _out_ptr(out, self.nvox, stream)
        self._check(self._L.tvs_initial_fbp(self._h, C.byref(prm), p, d, st), "tvs_initial_fbp")
        _settle(out, wait)
        return out

    def initial_fbp_noalloc(self, n_angles, median_radius=2, t_bin_mm=0.0, clip_negative=True,
                            out=None, stream=None):
        """initial_fbp through tvs_initial_fbp_noalloc: the library's fixed
        per-device workspace instead of allocations; with a device `out` the
        work is queued on torch's current stream (or waited for, when that is
        torch's default stream, whose null handle names the context's stream)."""
        prm = FbpParams(int(n_angles), int(median_radius), float(t_bin_mm), int(bool(clip_negative)), 0)
        if out is None:
            out = np.zeros(self.nvox, np.float32)
        p, d, st, wait = _out_ptr(out, self.nvox, stream)
        self._check(self._L.tvs_initial_fbp_noalloc(self._h, C.byref(prm), p, d, st),
                    "tvs_initial_fbp_noalloc")
        _settle(out, wait)
        return out

    def hull_detect(self, wepl_in_mm=1.0, wepl_out_mm=0.0, min_in=1, max_out=0,
                    mask_image=False, stream=None):
        """Hull of the object from the straight entry-exit lines of the loaded
        histories (tvs_hull_detect): space modelling (lines of WEPL >=
        wepl_in_mm count their voxels) and space carving (lines below
        wepl_out_mm carve them); returns the uint8 mask (x fastest).  With
        mask_image the context image is multiplied by it."""
        prm = HullParams(float(wepl_in_mm), float(wepl_out_mm), int(min_in), int(max_out),
                         int(bool(mask_image)), 0)
        out = np.zeros(self.nvox, np.uint8)
        self._check(self._L.tvs_hull_detect(self._h, C.byref(prm), C.c_void_p(out.ctypes.data), 0,
                                            _stream_handle(stream)), "tvs_hull_detect")
        return out

    def stats(self) -> dict:
        s = Stats()
        self._check(self._L.tvs_get_stats(self._h, C.byref(s)), "tvs_get_stats")
        return {n: getattr(s, n) for n, _ in Stats._fields_}

    def step_log(self) -> list:
        n = C.c_int64(0)
        self._check(self._L.tvs_get_step_log(self._h, None, 0, C.byref(n)), "tvs_get_step_log")
        buf = (StepLog * max(n.value, 1))()
        self._check(self._L.tvs_get_step_log(self._h, buf, n.value, C.byref(n)),
                    "tvs_get_step_log")
        return [{f: getattr(r, f) for f, _ in StepLog._fields_} for r in buf[:n.value]]

    def debug_rows(self, first, count, cap=None):
        """(row_nnz int64[count], idx int32[], chord float32[], norm2 float32[count])."""
        rn = np.zeros(max(count, 1), np.int64)
        n2 = np.zeros(max(count, 1), np.float32)
        if cap is None:
            self._L.tvs_debug_rows(self._h, first, count, rn.ctypes.data_as(C.POINTER(C.c_int64)),
                                   None, None, n2.ctypes.data_as(_FP), 0)
            cap = int(rn[:count].sum())
        idx = np.zeros(max(cap, 1), np.int32)
        ch = np.zeros(max(cap, 1), np.float32)
        rc = self._L.tvs_debug_rows(self._h, first, count, rn.ctypes.data_as(C.POINTER(C.c_int64)),
                                    idx.ctypes.data_as(C.POINTER(C.c_int32)), ch.ctypes.data_as(_FP),
                                    n2.ctypes.data_as(_FP), cap)
        self._check(rc, "tvs_debug_rows")
        tot = int(rn[:count].sum())
        return rn[:count], idx[:tot], ch[:tot], n2[:count]


def _info(i: RequestInfo) -> dict:
    return {f: getattr(i, f) for f, _ in RequestInfo._fields_}


class Server:
    """Continuous-batching server (tvs_server): FIFO admission by HBM budget and
    slots, one context and stream per running request."""

    def __init__(self, *, device=0, max_active=3, hbm_budget_bytes=0, chunk_histories=0,
                 simulate=False, sim_ns_per_history_cycle=0.0):
        self._L = load_library()
        cfg = ServerConfig()
        self._L.tvs_server_config_default(C.byref(cfg))
        cfg.device = int(device)
        cfg.max_active = int(max_active)
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        if chunk_histories:
            cfg.chunk_histories = int(chunk_histories)
        cfg.simulate = int(bool(simulate))
        cfg.sim_ns_per_history_cycle = float(sim_ns_per_history_cycle)
        h = C.c_void_p()
        rc = self._L.tvs_server_create(C.byref(cfg), C.byref(h))
        if rc != TVS_OK:
            raise TvsError(rc, "tvs_server_create: " + self._L.tvs_strerror(rc).decode())
        self._h = h
        self._keep = {}
        self._grids = {}

    def _request(self, grid, hist, lam, N, alpha, K, block_size, path_mode, seed, x0, variant,
                 tv_check):
        n = len(hist["ex"])
        arrs = {k: np.ascontiguousarray(hist[k], dtype=np.float32) for k in HIST_FIELDS}
        hs = Histories(*[C.c_void_p(arrs[k].ctypes.data) for k in HIST_FIELDS])
        v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        prm = Params(float(lam), int(N), float(alpha), int(bool(tv_check)), v, 0.0,
                     int(seed) & (2**64 - 1), 0.5)
        x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float32)
        req = Request(grid_struct(grid), int(block_size),
                      PATH_MODES[path_mode] if isinstance(path_mode, str) else int(path_mode),
                      prm, int(K), 0, n, hs, None if x0a is None else C.c_void_p(x0a.ctypes.data))
        return req, (arrs, x0a)

    def footprint(self, grid, hist, **kw):
        req, _ = self._request(grid, hist, kw.get("lam", 1e-4), kw.get("N", 1),
                               kw.get("alpha", 0.5), kw.get("K", 1), kw.get("block_size", 3200),
                               kw.get("path_mode", "otf"), 0, None, "ntvs", False)
        return int(self._L.tvs_server_footprint(self._h, C.byref(req)))

    def submit(self, grid, hist, *, lam, N, alpha, K, block_size=3200, path_mode="otf", seed=0,
               x0=None, variant="ntvs", tv_check=False):
        req, keep = self._request(grid, hist, lam, N, alpha, K, block_size, path_mode, seed, x0,
                                  variant, tv_check)
        rid = C.c_int64()
        rc = self._L.tvs_server_submit(self._h, C.byref(req), C.byref(rid))
        if rc != TVS_OK:
            raise TvsError(rc, "tvs_server_submit: " + self._L.tvs_strerror(rc).decode())
        self._keep[rid.value] = keep   # histories are borrowed until the request is done
        self._grids[rid.value] = int(grid.nx) * int(grid.ny) * int(grid.nz)
        return rid.value

    def query(self, rid):
        info = RequestInfo()
        rc = self._L.tvs_server_query(self._h, int(rid), C.byref(info))
        if rc != TVS_OK:
            raise TvsError(rc, "tvs_server_query")
        return _info(info)

    def wait(self, rid):
        """(image or None, info dict); the request's status is info['status']."""
        nv = self._grids[rid]
        img = np.zeros(nv, np.float32)
        info = RequestInfo()
        rc = self._L.tvs_server_wait(self._h, int(rid), img.ctypes.data_as(_FP), nv,
                                     C.byref(info))
        self._keep.pop(rid, None)
        return (img if rc == TVS_OK else None), _info(info)

    def counters(self):
        c = ServerCounters()
        self._L.tvs_server_get_counters(self._h, C.byref(c))
        return {f: getattr(c, f) for f, _ in ServerCounters._fields_}

    def close(self):
        if getattr(self, "_h", None):
            self._L.tvs_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
