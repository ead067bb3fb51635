"""Image-quality measures (arXiv 1803.01112, Section IV): total variation,
7 mm ROI statistics, RSP error; and the study summary.

Pinned by: zero TV and ROI spread on constant images, the closed form of a
step edge, agreement with the oracle's TV on random images, the number of
voxel centres in a 7 mm circle counted by brute force, ROI means of images
built from the phantom's own insert map, and the sign and scale of the RSP
error.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1803_01112_amd import quality, synth
from paper_1803_01112_amd.synth import Grid

G3 = Grid(9, 7, 3, 1.0, 1.0, 2.5, 0, 0, 0)


def test_tv_constant_and_step_edge():
    assert quality.total_variation(np.full(G3.nvox, 2.5), G3) == 0.0
    for h in (1.0, -0.75):
        x = np.zeros((G3.nz, G3.ny, G3.nx))
        x[:, :, 5:] = h
        assert quality.total_variation(x.ravel(), G3) == pytest.approx(abs(h) * G3.ny * G3.nz,
                                                                      rel=1e-15)
        z = np.zeros((G3.nz, G3.ny, G3.nx))
        z[2:, :, :] = h
        assert quality.total_variation(z.ravel(), G3) == 0.0


def test_tv_matches_oracle_on_random_images():
    rng = np.random.default_rng(1)
    for g in (G3, Grid(16, 11, 2, 1.0, 1.0, 2.5, 0, 0, 0)):
        x = rng.normal(1.0, 0.2, g.nvox)
        assert quality.total_variation(x, g) == pytest.approx(oracle.tv(g, x), rel=1e-12)


def test_roi_voxel_count_brute_force():
    g = synth.centered_grid(64, 64, 1, 1.0, 1.0, 2.5)
    # a circle centred on a voxel centre: the integer points within 3.5 voxels
    cx = g.ox + 30.5 * g.vx
    cy = g.oy + 20.5 * g.vy
    want = sum(1 for i in range(-4, 5) for j in range(-4, 5) if i * i + j * j <= 3.5 * 3.5)
    assert int(quality.roi_mask(g, cx, cy).sum()) == want == 37
    # and its area on a fine grid approaches pi r^2
    f = synth.centered_grid(400, 400, 1, 0.05, 0.05, 1.0)
    area = quality.roi_mask(f, 0.0, 0.0).sum() * 0.05 * 0.05
    assert area == pytest.approx(math.pi * 3.5 ** 2, rel=2e-3)


def test_roi_stats_on_the_phantom_map():
    w = synth.workload("vol200")
    g, ph = w.grid, w.phantom
    truth = synth.truth_image(g, ph).astype(np.float64)
    m = quality.measure(truth, g, ph)
    assert all(r > 3.5 + 0.75 for _, _, r, _ in ph.inserts)      # 6.1 mm inserts
    for q, (cx, cy, r, rsp) in zip(m["rois"], ph.inserts):
        # a 7 mm ROI lies inside an insert of radius r >= 3.5 mm only when
        # r > 3.5 + half a voxel diagonal; then it sees the insert alone
        if r > 3.5 + 0.75:
            assert q["mean"] == pytest.approx(rsp, rel=1e-6)
            assert q["std"] == pytest.approx(0.0, abs=1e-6)
            assert q["err_pct"] == pytest.approx(0.0, abs=1e-4)
        assert q["n"] > 0


def test_roi_stats_known_values():
    g = synth.centered_grid(32, 32, 3, 1.0, 1.0, 2.5)
    v = np.zeros((3, 32, 32))
    v[1] = 2.0
    X, Y = quality.voxel_centres_xy(g)
    v[1][X > 0] = 4.0                  # the ROI at the origin sees half 2, half 4
    st = quality.roi_stats(v.ravel(), g, 0.0, 0.0)
    m = quality.roi_mask(g, 0.0, 0.0)
    n_hi = int((m & (X > 0)).sum())
    n_lo = int(m.sum()) - n_hi
    mean = (2.0 * n_lo + 4.0 * n_hi) / (n_lo + n_hi)
    assert st["mean"] == pytest.approx(mean, rel=1e-15)
    var = (n_lo * (2.0 - mean) ** 2 + n_hi * (4.0 - mean) ** 2) / (n_lo + n_hi)
    assert st["std"] == pytest.approx(math.sqrt(var), rel=1e-12)
    # another slice is read only when asked
    assert quality.roi_stats(v.ravel(), g, 0.0, 0.0, slice_index=0)["mean"] == 0.0


def test_rsp_error_sign_and_scale():
    assert quality.rsp_error_pct(1.01, 1.0) == pytest.approx(1.0)
    assert quality.rsp_error_pct(0.57, 0.6) == pytest.approx(-5.0)


def test_paper_grid_fits_one_batch_and_summary_reads_the_right_cycle():
    st = quality.paper_grid(4)
    assert len(st) <= 32
    assert {s["study"] for s in st} == {"N", "alpha", "lambda", "repeat"}
    recs = []
    for s in range(len(st)):
        for k in range(1, 13):
            recs.append(dict(setting=s, cycle=k, tv=float(100 * s + k),
                             rois=[dict(mean=1.0 + 0.01 * s, std=0.1 * k, err_pct=float(k),
                                        rsp_true=1.0),
                                   dict(mean=0.5, std=0.0, err_pct=1e4, rsp_true=0.0012)]))
    out = quality.summarize(recs, st)
    for s, row in enumerate(out["rows"]):
        want = st[s].get("read_cycle", 12)
        assert row["cycle"] == want
        assert row["tv"] == 100 * s + want
        assert row["tv_first_cycles"] == [100 * s + c for c in (1, 2, 3, 4)]
        assert row["abs_err_pct"] == float(want)          # the air insert is left out
        assert row["err_pct"] == [float(want), 1e4]
    assert out["repeat_roi_mean_spread"] is not None
