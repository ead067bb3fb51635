"""Image-quality measures of reconstructed RSP images and a parameter-study
runner over the batched sweep.

The measures follow the paper's analysis (arXiv 1803.01112, Section IV):

* total variation of the image: the local variations added over every voxel,
  read (as everywhere in this package) as 2-D isotropic forward differences
  within each slice, a difference past the last row or column being zero;
* mean and standard deviation of the RSP in a circular region of interest
  (ROI) of 7 mm diameter centred in each insert: the voxels whose centres lie
  within the circle, in one slice (the paper analyses the central slice);
* RSP error of an ROI mean: its percentage difference from the insert's true
  RSP.

The study runner advances many (lambda, N, alpha) settings together through
`Context.iterate_batch` and measures every setting's image after each cycle,
so the paper's parameter-space studies (TV and noise against N, alpha,
lambda and repeated random draws) can be rerun on the synthetic phantoms.
These are host-side measurements of images the library returns; none of the
reconstruction runs here.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

ROI_DIAMETER_MM = 7.0
AIR_RSP_LIMIT = 0.1     # inserts below this true RSP are left out of mean errors


def as_volume(img, grid) -> np.ndarray:
    """Image as a (nz, ny, nx) float64 array (x fastest, the ABI's order)."""
    a = np.asarray(img, dtype=np.float64).reshape(int(grid.nz), int(grid.ny), int(grid.nx))
    return a


def total_variation(img, grid) -> float:
    """Sum over all voxels of sqrt(dx^2 + dy^2), forward differences in x and
    y within each slice (zero past the last column / row)."""
    v = as_volume(img, grid)
    dx = np.zeros_like(v)
    dy = np.zeros_like(v)
    dx[:, :, :-1] = v[:, :, 1:] - v[:, :, :-1]
    dy[:, :-1, :] = v[:, 1:, :] - v[:, :-1, :]
    return float(np.sum(np.sqrt(dx * dx + dy * dy)))


def voxel_centres_xy(grid):
    """Centres (x, y) in mm of the voxels of one slice, each (ny, nx)."""
    x = float(grid.ox) + (np.arange(int(grid.nx)) + 0.5) * float(grid.vx)
    y = float(grid.oy) + (np.arange(int(grid.ny)) + 0.5) * float(grid.vy)
    return np.meshgrid(x, y)


def roi_mask(grid, cx, cy, diameter=ROI_DIAMETER_MM) -> np.ndarray:
    """(ny, nx) mask of the voxels whose centres lie within the circle."""
    X, Y = voxel_centres_xy(grid)
    r = 0.5 * float(diameter)
    return (X - cx) ** 2 + (Y - cy) ** 2 <= r * r


def roi_stats(img, grid, cx, cy, diameter=ROI_DIAMETER_MM, slice_index=None) -> dict:
    """Mean, standard deviation (population) and voxel count of the RSP in a
    circular ROI of one slice (default: the central slice)."""
    v = as_volume(img, grid)
    k = int(grid.nz) // 2 if slice_index is None else int(slice_index)
    m = roi_mask(grid, cx, cy, diameter)
    vals = v[k][m]
    if vals.size == 0:
        return dict(mean=float("nan"), std=float("nan"), n=0)
    return dict(mean=float(vals.mean()), std=float(vals.std()), n=int(vals.size))


def rsp_error_pct(mean, true_rsp) -> float:
    """Percentage difference of an ROI mean from the true RSP."""
    return 100.0 * (float(mean) - float(true_rsp)) / float(true_rsp)


def measure(img, grid, phantom, slice_index=None) -> dict:
    """TV of the image and, per insert of the phantom, the ROI statistics
    and RSP error."""
    rois = []
    for cx, cy, _r, rsp in phantom.inserts:
        st = roi_stats(img, grid, cx, cy, slice_index=slice_index)
        st.update(rsp_true=float(rsp), err_pct=rsp_error_pct(st["mean"], rsp))
        rois.append(st)
    return dict(tv=total_variation(img, grid), rois=rois)


def run_study(ctx, grid, phantom, x0, settings, cycles, measure_every=1) -> list:
    """Advances all settings together (one batched sweep per cycle) from the
    initial image x0 and measures every setting's image after every
    `measure_every`-th cycle and after the last.  Returns one record per
    (setting, measured cycle)."""
    ctx.set_image(x0)
    out = []
    for k in range(1, int(cycles) + 1):
        ctx.iterate_batch(1, settings)
        if k % int(measure_every) == 0 or k == int(cycles):
            for s, st in enumerate(settings):
                img = ctx.get_batch_image(s)
                rec = dict(setting=s, cycle=k, lam=st["lam"], N=st["N"], alpha=st["alpha"],
                           seed=st.get("seed", 0))
                rec.update(measure(img, grid, phantom))
                out.append(rec)
    return out


def paper_grid(n_seeds=4, base_seed=1803):
    """Settings of the paper's studies that a batch can hold (up to 32):
    N in {1, 3, 5, 6, 12} at alpha 0.75 (TV and noise against N), alpha in
    {0.5, 0.65, 0.85, 0.95} at N = 5 (against alpha), lambda in {1.5e-4,
    2e-4} at N = 5, alpha = 0.75 (the equal-accuracy pairs are read at cycles
    8 and 6), and n_seeds repeats of N = 5, alpha = 0.75 with other seeds
    (spread of the random ell draws); lambda = 1e-4 unless stated."""
    out = []
    for N in (1, 3, 5, 6, 12):
        out.append(dict(lam=1e-4, N=N, alpha=0.75, seed=base_seed, study="N"))
    for a in (0.5, 0.65, 0.85, 0.95):
        out.append(dict(lam=1e-4, N=5, alpha=a, seed=base_seed, study="alpha"))
    for lam, k in ((1.5e-4, 8), (2e-4, 6)):
        out.append(dict(lam=lam, N=5, alpha=0.75, seed=base_seed, study="lambda", read_cycle=k))
    for q in range(n_seeds):
        out.append(dict(lam=1e-4, N=5, alpha=0.75, seed=base_seed + 1 + q, study="repeat"))
    return out


def summarize(records, settings) -> dict:
    """Per setting: TV, mean of the ROI standard deviations, the RSP errors
    and their mean magnitude over the inserts other than air (a percentage
    of 0.0012 says little) at its read cycle (its `read_cycle`, else the
    last measured), the
    TV after each of the first four cycles, and, for the repeats of one
    setting, the spread (standard deviation over seeds) of each ROI mean."""
    last, tv_by_cycle = {}, {}
    for r in records:
        want = settings[r["setting"]].get("read_cycle")
        if want is not None:
            if r["cycle"] == want:
                last[r["setting"]] = r
        elif r["setting"] not in last or r["cycle"] >= last[r["setting"]]["cycle"]:
            last[r["setting"]] = r
        if r["cycle"] <= 4:
            tv_by_cycle.setdefault(r["setting"], {})[r["cycle"]] = r["tv"]
    rows = []
    for s, st in enumerate(settings):
        r = last[s]
        rows.append(dict(study=st.get("study", ""), lam=st["lam"], N=st["N"], alpha=st["alpha"],
                         seed=st.get("seed", 0), cycle=r["cycle"], tv=r["tv"],
                         roi_std=float(np.mean([q["std"] for q in r["rois"]])),
                         err_pct=[q["err_pct"] for q in r["rois"]],
                         abs_err_pct=float(np.mean([abs(q["err_pct"]) for q in r["rois"]
                                                    if q["rsp_true"] >= AIR_RSP_LIMIT] or [np.nan])),
                         tv_first_cycles=[tv_by_cycle.get(s, {}).get(c) for c in (1, 2, 3, 4)]))
    rep = [s for s, st in enumerate(settings)
           if st.get("study") == "repeat" or (st.get("study") == "N" and st["N"] == 5)]
    spread = None
    if len(rep) > 1:
        means = np.array([[q["mean"] for q in last[s]["rois"]] for s in rep])
        spread = [float(v) for v in means.std(axis=0)]
    return dict(rows=rows, repeat_roi_mean_spread=spread)


def main(argv=None):
    ap = argparse.ArgumentParser(description="parameter study on a synthetic phantom")
    ap.add_argument("--workload", default="vol200")
    ap.add_argument("--n-hist", type=int, default=None)
    ap.add_argument("--cycles", type=int, default=12)
    ap.add_argument("--block", type=int, default=3200)
    ap.add_argument("--path-mode", default="f32")
    ap.add_argument("--seeds", type=int, default=4)
    ap.add_argument("--initial", default="flat", choices=("flat", "fbp"),
                    help="start from the hull-masked flat image or from the FBP initial "
                         "iterate with a radius-2 median (tvs_initial_fbp)")
    ap.add_argument("--out", default=None, help="write the records as JSON here")
    args = ap.parse_args(argv)

    import torch
    from . import synth, tvs
    w = synth.workload(args.workload, n_hist=args.n_hist)
    h = w.histories()
    dev = {k: torch.from_numpy(v).to("cuda:0") for k, v in h.items()}
    settings = paper_grid(args.seeds)
    ctx = tvs.Context(w.grid, block_size=args.block, path_mode=args.path_mode)
    ctx.load_histories(dev)
    if args.initial == "fbp":
        x0 = ctx.initial_fbp(w.n_angles, median_radius=2)
    else:
        x0 = w.initial_image()
    x0_measure = measure(x0, w.grid, w.phantom)
    t0 = time.perf_counter()
    recs = run_study(ctx, w.grid, w.phantom, x0, settings, args.cycles)
    dt = time.perf_counter() - t0
    ctx.close()
    summ = summarize(recs, settings)
    summ.update(workload=w.name, n_hist=w.n_hist, cycles=args.cycles, settings=len(settings),
                seconds=dt, initial=args.initial, initial_measure=x0_measure)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(dict(summary=summ, records=recs), fh)
    print(json.dumps(summ))
    return 0


if __name__ == "__main__":
    sys.exit(main())
