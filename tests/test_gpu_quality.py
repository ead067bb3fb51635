"""GPU: the parameter-study runner (batched sweep, one cycle per call, every
image measured after every cycle) against the same settings reconstructed
one at a time, and its images against the oracle's.

Image-quality measures follow arXiv 1803.01112, Section IV (TV, 7 mm ROI
mean/std, RSP error).  The measures of a batched image must equal those of
the setting's own reconstruction (images within 1e-5, the two GPU runs
differing only in the order of float atomics), and the oracle's image must
give the same measures within the 1e-4 image tolerance.
"""
import numpy as np
import pytest

import oracle
from paper_1803_01112_amd import quality, synth, tvs

pytestmark = pytest.mark.gpu

SETTINGS = [dict(lam=0.02, N=1, alpha=0.75, seed=7, study="N"),
            dict(lam=0.02, N=5, alpha=0.75, seed=7, study="N"),
            dict(lam=0.02, N=5, alpha=0.5, seed=7, study="alpha"),
            dict(lam=0.03, N=5, alpha=0.75, seed=7, study="lambda", read_cycle=2),
            dict(lam=0.02, N=5, alpha=0.75, seed=8, study="repeat")]
CYCLES = 3


def close_measures(a, b, e, nvox):
    """Measures of two images that differ by at most e per voxel: ROI means
    by e, ROI standard deviations by 2e, TV by 4e per voxel."""
    assert a["tv"] == pytest.approx(b["tv"], abs=4.0 * e * nvox)
    for qa, qb in zip(a["rois"], b["rois"]):
        assert qa["n"] == qb["n"]
        assert qa["mean"] == pytest.approx(qb["mean"], abs=e)
        assert qa["std"] == pytest.approx(qb["std"], abs=2.0 * e)


def test_study_matches_single_runs_and_oracle():
    w = synth.workload("slice64", n_hist=24_000)
    h = w.histories()
    g, ph = w.grid, w.phantom
    x0 = w.initial_image()
    print("study: slice64 24000 histories, 5 settings, 3 cycles", flush=True)
    with tvs.Context(g, block_size=64, mlp_step_mm=2.0, path_mode="f32") as ctx:
        ctx.load_histories(h)
        recs = quality.run_study(ctx, g, ph, x0, SETTINGS, CYCLES)
        assert len(recs) == CYCLES * len(SETTINGS)
        by = {(r["setting"], r["cycle"]): r for r in recs}
        for q, st in enumerate(SETTINGS):
            ctx.set_image(x0)
            for k in range(1, CYCLES + 1):
                ctx.iterate(1, st["lam"], st["N"], st["alpha"], seed=st["seed"])
                img = ctx.get_image()
                e = 1e-5 * max(float(np.max(np.abs(img))), 0.1)
                close_measures(by[(q, k)], quality.measure(img, g, ph), e, g.nvox)
    rows = oracle.build_rows(g, h, 2.0)
    for q in (1, 2):
        st = SETTINGS[q]
        S = oracle.Superiorizer(g, rows, x0, 64)
        S.iterate(CYCLES, st["lam"], st["N"], st["alpha"], seed=st["seed"])
        e = 1e-4 * max(float(np.max(np.abs(S.x))), 0.1)
        close_measures(by[(q, CYCLES)], quality.measure(S.x, g, ph), e, g.nvox)
    summ = quality.summarize(recs, SETTINGS)
    assert [r["cycle"] for r in summ["rows"]] == [3, 3, 3, 2, 3]
    assert len(summ["repeat_roi_mean_spread"]) == len(ph.inserts)
