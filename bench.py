"""Benchmark of the TVS proton-CT hot path on one MI355X.

A step is one TVS cycle of NTVS (arXiv 1803.01112, Appendix C): N
perturbation steps followed by one DROP feasibility sweep over every
history; the metric is histories processed per second per cycle.

Default workload (the largest single-GPU configuration): 256x256x32 voxels
of 1x1x2.5 mm, a 192 mm cylinder phantom with six inserts, 60M synthetic
histories at 360 angles, DROP blocks of 3200 histories (18,750 per sweep),
lambda = 1e-4, N = 5, alpha = 0.75, TV check off, rows (MLP + voxel walk)
formed on the fly inside every sweep.  Beside it, on the same histories:
the path stores (float32 chords, float16 chords, the 6-byte fixed-point
store) and the check-on cycle.  Further legs: the store forms' image error
against the oracle on the two-slice sub-problem, the 24-setting batched
parameter study on the 200x200x16 volume's 20M histories, and a stream of
serving requests.  Inputs are generated (seeded), copied to HBM and loaded
before any timed region starts.

HBM accounting: algorithmic bytes of one sweep are 16 B per history (WEPL,
||a||^2, row offset) plus (4 + chord bytes) per row entry of a path store,
or 52 B per history (the 13 float32 streams) on the fly, read once.

Prints one JSON line.  Only one GPU is supported: --gpus above 1 exits.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# float64 operations of one MLP vertex (scattering moments, two 2x2
# conditionings, vertex position and its segment's voxel walk), the count of
# the hot-path scope's measurement plan
FP64_FLOPS_PER_VERTEX = 250.0
CHORD_BYTES = {"otf": 4, "f32": 4, "f16": 2, "q16": 2}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def sweep_bytes(H, nnz, mode):
    """Algorithmic HBM bytes of the DROP chain in one sweep: 16 B per history
    (WEPL, ||a||^2, row offset) and (4 + chord bytes) per row entry, read
    once.  On the fly the entries the row formation wrote (4-byte tag +
    float32 chord) are what the chain reads; the history streams themselves
    are 52 B per history (on_the_fly_stream_bytes)."""
    return 16.0 * H + (4.0 + CHORD_BYTES[mode]) * nnz


# sources of each measured kernel: a counter record taken on other sources
# no longer describes the kernel
KERNEL_SOURCES = {
    "k_drop_tile": ("paper_1803_01112_amd/csrc/drop.hip", "paper_1803_01112_amd/csrc/device_common.hpp",
                    "paper_1803_01112_amd/csrc/tvs_internal.hpp"),
    "k_rows_fill_tiled": ("paper_1803_01112_amd/csrc/rows.hip", "paper_1803_01112_amd/csrc/tvs_internal.hpp"),
}


def source_hash(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from a committed counter record
    (profiles/*_counters.md: FETCH_SIZE and WRITE_SIZE passes, each scaled
    by what it reads for a copy of known size), or None when there is no
    record for this kernel and workload taken on the current sources."""
    import glob
    want = source_hash(kernel)
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_counters.md"))):
        with open(path) as fh:
            for line in fh:
                if not line.startswith("counter-record: "):
                    continue
                rec = json.loads(line[len("counter-record: "):])
                if (rec.get("kernel_family") == kernel and rec.get("workload") == workload
                        and rec.get("source_sha256") == want):
                    return rec["bytes_per_launch"]
    return None


def mlp_vertices(h, step):
    u = np.stack([h["ux"], h["uy"]]).astype(np.float64)
    u /= np.hypot(u[0], u[1])
    L = (h["qx"] - h["ex"]) * u[0] + (h["qy"] - h["ey"]) * u[1]
    J = np.maximum(np.ceil(L / step), 1.0)
    return float(np.sum(np.where(L > 0, J - 1, 0)))


def percentiles(lat):
    return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
            "cycles": len(lat)}


def timed_cycles(torch, ctx, K, kw):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.iterate(K, **kw)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def latency(torch, ctx, n, kw):
    """Per-cycle wall time, each cycle synchronised on its own (ms)."""
    out = []
    for _ in range(n):
        out.append(1e3 * timed_cycles(torch, ctx, 1, kw))
    return out


def run_form(tvs, torch, w, dev_hist, x0, args, mode, K, W, n_lat, check=False, block=None):
    """Loads the histories in path mode `mode` (DROP blocks of `block`
    histories, default the benchmark's), runs W untimed and K timed cycles,
    then n_lat cycles one at a time; returns figures and stats."""
    block = block or args.block
    ctx = tvs.Context(w.grid, block_size=block, path_mode=mode,
                      time_sample=args.time_sample)
    t0 = time.perf_counter()
    ctx.load_histories(dev_hist)
    torch.cuda.synchronize()
    load_s = time.perf_counter() - t0
    ctx.set_image(x0)
    tune = None
    if args.tune:
        # the library's launch-shape tuner (on the fly also the share of row
        # chunks formed at full occupancy); it restores the image
        tune = ctx.autotune(args.lam)
        log(f"{mode}: tuned {tune['tile_threads']} threads, sweep kernel {tune['sweep_kernel']}, "
            f"full-occupancy row chunks {tune['fill_wide_pct']} %")
    kw = dict(lam=args.lam, N=args.N, alpha=args.alpha, tv_check=check, seed=args.seed)
    if W > 0:
        ctx.iterate(W, **kw)
    dt = timed_cycles(torch, ctx, K, kw)
    st = ctx.stats()
    lat = latency(torch, ctx, n_lat, kw) if n_lat > 0 else []
    steps = ctx.step_log() if check else None
    ctx.close()
    H = w.n_hist
    T = math.ceil(H / block)
    sweep_ms = st["drop_ms_total"] / max(st["drop_launches"], 1)
    ns = max(st["k_samples"], 1)
    out = dict(value=H * K / dt, unit="histories/s", ms_per_step=1e3 * dt / K,
               load_s=load_s, nnz=st["nnz"],
               phases_ms_per_cycle={"tv": st["tv_ms_total"] / max(st["cycles_timed"], 1),
                                    "sweep": st["sweep_ms_total"] / max(st["cycles_timed"], 1),
                                    "rows": st["rows_ms_total"] / max(st["cycles_timed"], 1),
                                    "drop": sweep_ms},
               block_size=block, drop_steps=T + 1,
               drop_step_us=1e3 * sweep_ms / (T + 1),
               drop_launch_us=1e3 * st["k1_ms_total"] / ns)
    b = sweep_bytes(H, st["nnz"], mode)
    out["hbm"] = dict(algorithmic_bytes_per_sweep=b,
                      gbs=b / (sweep_ms * 1e-3) / 1e9,
                      frac=b / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      what="algorithmic bytes of one sweep over the DROP chain's device time")
    if mode == "otf":
        out["hbm"]["on_the_fly_stream_bytes"] = 52.0 * H
    if tune is not None:
        out["tuned"] = dict(tile_threads=tune["tile_threads"], sweep_kernel=tune["sweep_kernel"],
                            fill_wide_pct=tune["fill_wide_pct"] if mode == "otf" else None)
    if lat:
        out["latency_ms"] = percentiles(lat)
    if steps is not None:
        tries = [r["tries"] for r in steps]
        out["check"] = dict(steps=len(steps), tries_total=int(sum(tries)),
                            tries_max=int(max(tries) if tries else 0),
                            accepted=int(sum(r["accepted"] for r in steps)))
    return out, st


def cpu_baseline(w, args, cores):
    """The oracle (plain float64 CPU code) on a bounded prefix of the same
    scan (1M histories by default), one cycle as the library runs it on the
    fly: rows formed (MLP + walk; OpenMP over histories on all host threads,
    and on one thread for a tenth of the prefix), then N TV steps and one
    DROP sweep (one thread).  The sweep alone and a cycle with the TV check
    are timed beside it, so the phases are reported separately."""
    import oracle
    n = args.cpu_sample
    h = w.histories(count=n)
    x0 = w.initial_image()
    oracle.set_threads(cores)
    t0 = time.perf_counter()
    rows = oracle.build_rows(w.grid, h, min(w.grid.vx, w.grid.vy))
    t_rows = time.perf_counter() - t0
    n1 = max(n // 10, 1)
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.build_rows(w.grid, {k: v[:n1] for k, v in h.items()}, min(w.grid.vx, w.grid.vy))
    t_rows1 = (time.perf_counter() - t0) * n / n1
    oracle.set_threads(cores)
    S = oracle.Superiorizer(w.grid, rows, x0, args.block)
    t0 = time.perf_counter()
    S.iterate(1, args.lam, args.N, args.alpha, seed=args.seed)
    t_cycle = time.perf_counter() - t0
    S0 = oracle.Superiorizer(w.grid, rows, x0, args.block)
    t0 = time.perf_counter()
    S0.iterate(1, args.lam, 0, args.alpha, seed=args.seed)
    t_sweep = time.perf_counter() - t0
    Sc = oracle.Superiorizer(w.grid, rows, x0, args.block)
    t0 = time.perf_counter()
    Sc.iterate(1, args.lam, args.N, args.alpha, tv_check=1, seed=args.seed)
    t_checked = time.perf_counter() - t0
    el = t_rows + t_cycle
    return dict(value=n / el, unit="histories/s", cores=cores, kind="oracle",
                single_thread_value=n / (t_rows1 + t_cycle),
                phases_s_per_cycle={"rows_mlp_walk_all_cores": t_rows,
                                    "rows_mlp_walk_one_thread": t_rows1,
                                    "tv_steps_and_drop_sweep_one_thread": t_cycle,
                                    "drop_sweep_one_thread": t_sweep,
                                    "tv_steps_one_thread": max(t_cycle - t_sweep, 0.0),
                                    "tv_steps_checked_one_thread": max(t_checked - t_sweep, 0.0)},
                sample=f"first {n} histories of the {w.name} scan ({w.n_hist}); one cycle: rows "
                       f"(MLP + walk) on {cores} threads, then N={args.N} TV steps and one DROP "
                       f"sweep on one thread ({el:.1f} s); the one-thread row time is measured "
                       f"on the first {n1} histories and scaled")


def precision_report(tvs, torch, args):
    """Image error of each path form against the oracle on the two-slice
    sub-problem of the 256x256x32 phantom (256x256x2 voxels of 1x1x2.5 mm,
    3.75M histories at 360 angles, B = 3200), K cycles at the benchmark's
    lambda, N, alpha: max and RMS of |x - x_oracle| / max(|x_oracle|, 0.1),
    and the largest change of a 7 mm insert ROI mean."""
    import oracle
    from paper_1803_01112_amd import quality, synth
    w = synth.workload("slab256", n_hist=args.precision_hist)
    h = w.histories()
    x0 = w.initial_image()
    K = args.precision_cycles
    kw = dict(lam=args.lam, N=args.N, alpha=args.alpha, seed=args.seed)
    t0 = time.perf_counter()
    rows = oracle.build_rows(w.grid, h, min(w.grid.vx, w.grid.vy))
    S = oracle.Superiorizer(w.grid, rows, x0, args.block)
    S.iterate(K, **kw)
    t_or = time.perf_counter() - t0
    del rows
    ref = S.x
    roi_ref = [q["mean"] for q in quality.measure(ref, w.grid, w.phantom)["rois"]]
    dev = {k: torch.from_numpy(v).to("cuda:0") for k, v in h.items()}
    out = dict(workload=f"{w.name}: {w.grid.nx}x{w.grid.ny}x{w.grid.nz}, {w.n_hist} histories",
               cycles=K, oracle_seconds=t_or, tolerance=1e-4, forms={})
    for form in ("f32", "q16", "f16", "otf"):
        with tvs.Context(w.grid, block_size=args.block, path_mode=form) as ctx:
            ctx.load_histories(dev)
            ctx.set_image(x0)
            ctx.iterate(K, **kw)
            x = ctx.get_image().astype(np.float64)
        e = np.abs(x - ref) / np.maximum(np.abs(ref), 0.1)
        roi = [q["mean"] for q in quality.measure(x, w.grid, w.phantom)["rois"]]
        out["forms"][form] = dict(max_rel=float(e.max()), rms_rel=float(np.sqrt(np.mean(e * e))),
                                  max_roi_mean_delta=float(np.max(np.abs(np.subtract(roi, roi_ref)))),
                                  meets_tolerance=bool(e.max() <= 1e-4))
        log(f"precision {form}: {out['forms'][form]}")
    return out


def batch_settings():
    """24 settings: lambda in {1e-4, 2e-4} x N in {1, 3, 6} x alpha in {0.5, 0.75, 0.85, 0.95}."""
    out = []
    for lam in (1e-4, 2e-4):
        for N in (1, 3, 6):
            for alpha in (0.5, 0.75, 0.85, 0.95):
                out.append(dict(lam=lam, N=N, alpha=alpha, seed=1803 + len(out)))
    return out


def run_batch(tvs, torch, args):
    """The 24-setting parameter study advanced together on the 200x200x16
    volume's 20M histories (one row stream per cycle for all settings),
    against the same store's single-setting cycle."""
    from paper_1803_01112_amd import synth
    w = synth.workload("vol200")
    log(f"batch leg: generating {w.n_hist} histories of {w.name}")
    h = w.histories()
    dev = {k: torch.from_numpy(v).to("cuda:0") for k, v in h.items()}
    del h
    x0 = torch.from_numpy(w.initial_image()).to("cuda:0")
    sets = batch_settings()
    S = len(sets)
    ctx = tvs.Context(w.grid, block_size=args.block, path_mode=args.batch_path)
    ctx.load_histories(dev)
    ctx.set_image(x0)
    # the plain single-setting cycle of the same store, for comparison
    kw = dict(lam=1e-4, N=3, alpha=0.75, seed=args.seed)
    ctx.iterate(1, **kw)
    dt1 = timed_cycles(torch, ctx, args.batch_steps, kw) / args.batch_steps
    ctx.set_image(x0)
    tune = ctx.autotune_batch(sets)                # threads x settings per LDS pass
    log(f"batch shape: {tune['threads']} threads, {tune['group']} settings per pass")
    ctx.iterate_batch(1, sets)                     # warm-up cycle (captures the graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.iterate_batch(args.batch_steps, sets)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.batch_steps
    st = ctx.stats()
    lat = []
    for _ in range(args.batch_latency):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.iterate_batch(1, sets)
        torch.cuda.synchronize()
        lat.append(1e3 * (time.perf_counter() - t0))
    ctx.close()
    del dev
    H = w.n_hist
    return dict(workload=f"{w.name}: 200x200x16, {H} histories", settings=S,
                value=H * S / dt, unit="history-settings/s", ms_per_cycle=1e3 * dt,
                device_ms_per_cycle=st["batch_ms_total"] / max(st["batch_cycles"], 1),
                latency_ms=percentiles(lat) if lat else None,
                single_setting=dict(value=H / dt1, ms_per_cycle=1e3 * dt1, N=3, alpha=0.75),
                speedup_vs_separate_runs=(S * dt1) / dt, path_mode=args.batch_path,
                shape=dict(threads=tune["threads"], settings_per_pass=tune["group"],
                           ms_per_block=tune["ms_per_block"],
                           candidates=[(c["threads"], c["group"], round(c["ms"], 5))
                                       for c in tune["candidates"]]))


def run_serving(tvs, args):
    """Poisson stream of reconstruction requests: grids drawn from 64x64x4 ..
    256x256x32, history counts log-uniform in [serve_hmin, serve_hmax], the
    paper's equal-accuracy (lambda, K) pairs, N in 1..6, alpha from the
    paper's grid; offered at fractions of the measured serial capacity."""
    from paper_1803_01112_amd import synth
    rng = np.random.default_rng(1803011124)
    grids = ["vol64", "vol128", "vol200", "vol256"]
    hmax = args.serve_hmax
    pools = {}
    for g in grids:
        w = synth.workload(g, n_hist=hmax)
        pools[g] = (w, w.histories(), w.initial_image())
        log(f"serving pool {g}: {hmax} histories")
    pairs = [(1e-4, 12), (1.5e-4, 8), (2e-4, 6)]
    reqs = []
    for q in range(args.serve_requests):
        g = grids[rng.integers(len(grids))]
        n = int(10 ** rng.uniform(np.log10(args.serve_hmin), np.log10(hmax)))
        lam, K = pairs[rng.integers(3)]
        reqs.append(dict(g=g, n=n, lam=lam, K=K, N=int(rng.integers(1, 7)),
                         alpha=float(rng.choice([0.5, 0.65, 0.75, 0.85, 0.95]))))
    work = sum(r["n"] * r["K"] for r in reqs)

    def sub(s, r):
        w, h, x0 = pools[r["g"]]
        hh = {k: v[:r["n"]] for k, v in h.items()}
        return s.submit(w.grid, hh, lam=r["lam"], N=r["N"], alpha=r["alpha"], K=r["K"],
                        path_mode=args.serve_path, x0=x0, seed=7)

    if args.serve_capacity > 0:
        # a capacity measured before (history-cycles/s of requests run one
        # at a time): long mixes skip the serial pass
        t_alone = work / args.serve_capacity
        log(f"serving: capacity given, {args.serve_capacity:.4g} history-cycles/s")
    else:
        with tvs.Server(max_active=1) as s:
            t0 = time.perf_counter()
            for q, r in enumerate(reqs):
                s.wait(sub(s, r))
                if (q + 1) % 20 == 0:
                    log(f"serving: {q + 1} of {len(reqs)} requests run one at a time")
            t_alone = time.perf_counter() - t0
        log(f"serving: {len(reqs)} requests one at a time in {t_alone:.1f} s")
    cap_rate = len(reqs) / t_alone
    out = dict(requests=len(reqs), histories=f"log-uniform in [{args.serve_hmin}, {hmax}]",
               history_cycles=work, serial_s=None if args.serve_capacity > 0 else t_alone,
               serial_value=work / t_alone, capacity_given=args.serve_capacity > 0,
               slots=args.serve_slots, path_mode=args.serve_path, loads={})
    for rho in [float(v) for v in args.serve_loads.split(",")]:
        gaps = rng.exponential(1.0 / (rho * cap_rate), len(reqs))
        with tvs.Server(max_active=args.serve_slots) as s:
            t0 = time.perf_counter()
            ids = []
            for q, (r, gap) in enumerate(zip(reqs, gaps)):
                time.sleep(gap)
                ids.append(sub(s, r))
                if (q + 1) % 20 == 0:
                    log(f"serving at load {rho}: {q + 1} of {len(reqs)} submitted")
            res = []
            for q, i in enumerate(ids):
                res.append(s.wait(i))
                if (q + 1) % 20 == 0:
                    log(f"serving at load {rho}: {q + 1} of {len(reqs)} done")
            dt = time.perf_counter() - t0
            c = s.counters()
        lat = np.array([i["done_ms"] - i["submit_ms"] for _, i in res])
        ok = sum(1 for _, i in res if i["status"] == 0)
        out["loads"][str(rho)] = dict(value=work / dt, unit="history-cycles/s", makespan_s=dt,
                                      p50_ms=float(np.percentile(lat, 50)),
                                      p99_ms=float(np.percentile(lat, 99)), completed=ok,
                                      peak_active=c["peak_active"],
                                      peak_gb=c["peak_bytes"] / 2**30)
        log(f"serving at load {rho}: {out['loads'][str(rho)]}")
    return out


def references(torch):
    """A STREAM-like copy on this device and a unique-address float atomic
    rate (the roofline keeps the published peak; these say what plain
    kernels reach here)."""
    src = torch.ones(512 << 20, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    n_at = 64 << 20
    acc = torch.zeros(n_at, dtype=torch.float32, device="cuda:0")
    idx = torch.arange(n_at, dtype=torch.int64, device="cuda:0")
    val = torch.ones(n_at, dtype=torch.float32, device="cuda:0")
    acc.index_add_(0, idx, val)
    e0.record()
    for _ in range(3):
        acc.index_add_(0, idx, val)
    e1.record()
    torch.cuda.synchronize()
    at_ms = e0.elapsed_time(e1) / 3
    del acc, idx, val
    return ({"copy_gbs": copy_gbs, "frac_of_published": copy_gbs / HBM_PEAK_GBS,
             "what": "device-to-device copy of 2 GiB, bytes read + written / time"},
            {"what": "torch index_add_, float32, 64M unique consecutive addresses",
             "lane_atomics_per_s": n_at / (at_ms * 1e-3), "ms": at_ms})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="vol256")
    ap.add_argument("--n-hist", type=int, default=None)
    ap.add_argument("--block", type=int, default=3200)
    ap.add_argument("--lam", type=float, default=1e-4)
    ap.add_argument("--N", type=int, default=5)
    ap.add_argument("--alpha", type=float, default=0.75)
    ap.add_argument("--seed", type=int, default=1803011121)
    ap.add_argument("--path-mode", default="otf")
    ap.add_argument("--time-sample", type=int, default=16,
                    help="kernel-stamped HIP events on the launch of every k-th DROP block")
    ap.add_argument("--latency-cycles", type=int, default=50)
    ap.add_argument("--forms", default="f32,f16,q16,q16@25600",
                    help="path-store forms timed beside (mode or mode@block size)")
    ap.add_argument("--form-steps", type=int, default=10)
    ap.add_argument("--form-latency", type=int, default=50)
    ap.add_argument("--legs", default="check,precision,batch,serve",
                    help="further legs: check, precision, batch, serve")
    ap.add_argument("--check-steps", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=1_000_000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="skip the library's launch-shape tuner before each timed form")
    ap.add_argument("--batch-path", default="f32")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--batch-latency", type=int, default=10)
    ap.add_argument("--serve-requests", type=int, default=40)
    ap.add_argument("--serve-hmin", type=int, default=1_000_000)
    ap.add_argument("--serve-hmax", type=int, default=8_000_000)
    ap.add_argument("--serve-slots", type=int, default=3)
    ap.add_argument("--serve-loads", default="0.5,0.8,0.95")
    ap.add_argument("--serve-path", default="q16")
    ap.add_argument("--serve-capacity", type=float, default=0.0,
                    help="serial capacity in history-cycles/s (skips the serial pass)")
    ap.add_argument("--fbp", action="store_true",
                    help="also time the initial iterate (FBP + median) and hull detection of "
                         "all histories")
    ap.add_argument("--precision-hist", type=int, default=3_750_000)
    ap.add_argument("--precision-cycles", type=int, default=3)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with a 256 MiB read + 256 MiB write kernel (scales the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--print-source-hash", action="store_true",
                    help="print the hash of each measured kernel's sources and exit")
    args = ap.parse_args()
    if args.print_source_hash:
        for k in KERNEL_SOURCES:
            print(k, source_hash(k))
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1803_01112_amd import synth, tvs

    tvs.load_library()
    legs = {l for l in args.legs.split(",") if l}
    w = synth.workload(args.workload, n_hist=args.n_hist)
    log(f"generating {w.n_hist} histories of {w.name}")
    t0 = time.perf_counter()
    h = w.histories()
    log(f"generated in {time.perf_counter() - t0:.1f} s; copying to HBM")
    dev = {k: torch.from_numpy(v).to("cuda:0") for k, v in h.items()}
    x0 = torch.from_numpy(w.initial_image()).to("cuda:0")
    torch.cuda.synchronize()
    step_mm = min(w.grid.vx, w.grid.vy)
    vertices = mlp_vertices(h, step_mm)
    fbp_h = h if args.fbp else None
    del h
    H = w.n_hist
    T = math.ceil(H / args.block)

    log(f"timing {args.path_mode}: warmup {args.warmup}, steps {args.steps}, "
        f"latency cycles {args.latency_cycles}")
    head, st = run_form(tvs, torch, w, dev, x0, args, args.path_mode, args.steps, args.warmup,
                        args.latency_cycles)
    log(f"{args.path_mode}: {head}")

    # dominant kernel of the timed region: the DROP step (one launch per
    # block, kernel-stamped events on every k-th block) or the row formation
    # on the second stream (events around every launch)
    nnz = st["nnz"]
    k1_ms = st["k1_ms_total"] / max(st["k_samples"], 1)
    if st["k_samples"] == 0:
        # no kernel-stamped launches (--time-sample 0): the chain's device
        # time per step stands in for the launch duration
        k1_ms = st["drop_ms_total"] / max(st["drop_launches"], 1) / (T + 1)
    rows_ms = st["rows_ms_total"] / max(st["rows_launches"], 1)
    per_cycle = {"k_drop_tile": k1_ms * (T + 1)}
    if args.path_mode == "otf":
        per_cycle["k_rows_fill_tiled"] = st["rows_ms_total"] / max(st["cycles_timed"], 1)
    dom = max(per_cycle, key=per_cycle.get)

    def roofline_of(kernel):
        if kernel == "k_rows_fill_tiled":
            launches = max(st["rows_launches"] / max(st["cycles_timed"], 1), 1)
            per_launch = FP64_FLOPS_PER_VERTEX * vertices / launches
            achieved = per_launch / (rows_ms * 1e-3) / 1e12
            r = dict(bound="alu", kernel=kernel, achieved=achieved, peak=FP64_PEAK_TFLOPS,
                     unit="TFLOP/s", frac=achieved / FP64_PEAK_TFLOPS, traffic=None,
                     avg_launch_ms=rows_ms, algorithmic_per_launch=per_launch,
                     unit_of_work=f"{FP64_FLOPS_PER_VERTEX:.0f} FP64 flops per MLP vertex, "
                                  f"{vertices / launches:.4g} vertices per launch")
        else:
            per_launch = sweep_bytes(H, nnz, args.path_mode) / T
            achieved = per_launch / (k1_ms * 1e-3) / 1e9
            r = dict(bound="hbm", kernel=kernel, achieved=achieved, peak=HBM_PEAK_GBS,
                     unit="GB/s", frac=achieved / HBM_PEAK_GBS, traffic=None,
                     avg_launch_ms=k1_ms, algorithmic_per_launch=per_launch,
                     unit_of_work="16 B per history + (4 + chord bytes) per entry of one block")
        r["traffic"] = measured_traffic(kernel, f"{w.name}/{H}/B{args.block}/{args.path_mode}")
        return r

    roof = roofline_of(dom)
    roof["per_cycle_ms"] = per_cycle
    # the other kernel of the cycle (on the fly the row formation runs beside
    # the chain on its own stream)
    others = {k: roofline_of(k) for k in per_cycle if k != dom}

    forms = {}
    for form in [f for f in args.forms.split(",") if f]:
        log(f"timing form {form}")
        mode, _, blk = form.partition("@")
        forms[form], _ = run_form(tvs, torch, w, dev, x0, args, mode, args.form_steps, 1,
                                  args.form_latency, block=int(blk) if blk else None)
        forms[form]["store_build_s"] = forms[form].pop("load_s")
        log(f"{form}: {forms[form]}")

    check = None
    if "check" in legs:
        log("timing the check-on cycle")
        check, _ = run_form(tvs, torch, w, dev, x0, args, args.path_mode, args.check_steps, 1, 0,
                            check=True)
        check["vs_check_off"] = check["value"] / head["value"]
        log(f"check on: {check}")

    fbp = None
    if fbp_h is not None:
        ctx = tvs.Context(w.grid, block_size=args.block)
        ctx.load_histories(dev)
        tms = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.initial_fbp(w.n_angles, median_radius=2)
            tms.append(time.perf_counter() - t0)
        # hull detection (space modelling on the same histories, every one
        # of which crosses the object), returned to the host
        hms = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hull = ctx.hull_detect(wepl_in_mm=1.0, min_in=1)
            hms.append(time.perf_counter() - t0)
        ctx.close()
        fbp = dict(ms=1e3 * min(tms), unit="ms per initial iterate", histories=H,
                   n_angles=w.n_angles, median_radius=2,
                   hull_ms=1e3 * min(hms), hull_voxels=int(hull.sum()))
        log(f"fbp: {fbp}")
        del fbp_h
    del dev
    torch.cuda.empty_cache()

    precision = None
    if "precision" in legs:
        log("precision leg")
        precision = precision_report(tvs, torch, args)
    batch = None
    if "batch" in legs:
        batch = run_batch(tvs, torch, args)
        log(f"batch: {batch}")
        torch.cuda.empty_cache()
    serving = None
    if "serve" in legs:
        log("serving leg")
        serving = run_serving(tvs, args)

    if args.copy_calibration:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.add(a, 1.0, out=b)
        torch.cuda.synchronize()
        log("copy calibration: 268435456 bytes read, 268435456 bytes written")
        del a, b
    hbm_measured, atomic_reference = references(torch)
    log(f"references: {hbm_measured} {atomic_reference}")

    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cpu = None if args.no_cpu else cpu_baseline(w, args, cores)

    out = {
        "metric": "proton histories/s per TVS iteration (MLP+DROP+TV)",
        "value": head["value"],
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.grid.nx}x{w.grid.ny}x{w.grid.nz} voxels of "
                               f"{w.grid.vx}x{w.grid.vy}x{w.grid.vz} mm, {w.diameter:.0f} mm "
                               f"cylinder with 6 inserts, {H} histories at {w.n_angles} angles",
                   "block_size": args.block, "blocks_per_sweep": T, "lambda": args.lam,
                   "N": args.N, "alpha": args.alpha, "tv_check": False,
                   "path_mode": args.path_mode, "nnz": nnz, "parallelism": "1 GPU"},
        "latency_ms": head.get("latency_ms"),
        "phases_ms_per_cycle": head["phases_ms_per_cycle"],
        "hbm": head["hbm"],
        "load_s": head["load_s"],
        "roofline": roof,
        "roofline_other_kernels": others,
        "hbm_measured": hbm_measured,
        "atomic_reference": atomic_reference,
        "forms": forms,
        "check": check,
        "precision": precision,
        "batch": batch,
        "serving": serving,
        "fbp": fbp,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
