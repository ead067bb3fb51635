"""Pins of the oracle's hull detection (space modelling and space carving on
each history's straight entry-exit line; the paper's preprocessing, Section
III-D, bounds the object before the MLP and cites, not gives, how).

Checked against what does not depend on the oracle's walk: voxel rows of
axis-aligned lines, brute-force sampling along random lines, and the
geometry of the cylinder phantom (chords of a convex object stay inside it;
lines that miss it carve only outside it)."""
import math

import numpy as np
import pytest

import oracle
from paper_1803_01112_amd import synth


lines = synth.line_histories


def test_axis_line_counts_its_voxel_row():
    g = synth.Grid(6, 5, 2, 1.0, 1.0, 1.0, 0.0, 0.0, 0.0)
    h = lines([[-1.0, 2.5, 0.5]], [[7.0, 2.5, 0.5]], [10.0])
    cin, cout = oracle.hull_counts(g, h, 1.0, 1.0)
    want = np.zeros(g.nvox, np.int32)
    want[[i + 6 * 2 for i in range(6)]] = 1            # row j = 2 of slice 0
    np.testing.assert_array_equal(cin, want)
    assert not cout.any()
    h = lines([[-1.0, 2.5, 0.5]], [[7.0, 2.5, 0.5]], [0.0])   # a miss carves the same row
    cin, cout = oracle.hull_counts(g, h, 1.0, 1.0)
    assert not cin.any()
    np.testing.assert_array_equal(cout, want)


def test_random_lines_match_sampling():
    g = synth.Grid(7, 6, 3, 1.0, 1.3, 0.8, -3.5, -3.9, -1.2)
    rng = np.random.default_rng(4)
    n = 40
    p0 = np.stack([rng.uniform(-5, 5, n), rng.uniform(-5, 5, n), rng.uniform(-1.5, 1.5, n)], 1)
    p1 = np.stack([rng.uniform(-5, 5, n), rng.uniform(-5, 5, n), rng.uniform(-1.5, 1.5, n)], 1)
    h = lines(p0, p1, np.full(n, 5.0))
    cin, _ = oracle.hull_counts(g, h, 1.0, 0.0)
    want = np.zeros(g.nvox, np.int64)
    t = (np.arange(200000) + 0.5) / 200000
    for a, b in zip(p0, p1):
        pts = a[None, :] + t[:, None] * (b - a)[None, :]
        ijk = np.floor((pts - [g.ox, g.oy, g.oz]) / [g.vx, g.vy, g.vz]).astype(np.int64)
        ok = np.all((ijk >= 0) & (ijk < [g.nx, g.ny, g.nz]), axis=1)
        ijk = ijk[ok]
        lin, cnt = np.unique(ijk[:, 0] + g.nx * (ijk[:, 1] + g.ny * ijk[:, 2]), return_counts=True)
        seen = np.zeros(g.nvox, bool)
        seen[lin] = True
        # voxels the line spends at least two samples in are crossed; the
        # walk may add corner grazes shorter than that
        sure = np.zeros(g.nvox, bool)
        sure[lin[cnt >= 2]] = True
        idx, ch, _ = oracle.walk_polyline(g, np.stack([a, b]))
        walked = np.zeros(g.nvox, bool)
        walked[idx] = True
        assert np.all(walked[sure])
        assert not np.any(walked & ~seen & (np.bincount(idx, ch, g.nvox) > 3e-5 * np.linalg.norm(b - a)))
        want += walked
    np.testing.assert_array_equal(cin, want)


def _disk_masks(g, R):
    """Voxels whose square meets the disk of radius R / lies inside radius r."""
    i = np.arange(g.nx)
    j = np.arange(g.ny)
    x0 = g.ox + i * g.vx
    y0 = g.oy + j * g.vy
    X0, Y0 = np.meshgrid(x0, y0)
    X1, Y1 = X0 + g.vx, Y0 + g.vy
    nearest = np.hypot(np.clip(0.0, X0, X1), np.clip(0.0, Y0, Y1))
    farthest = np.hypot(np.maximum(abs(X0), abs(X1)), np.maximum(abs(Y0), abs(Y1)))
    return (nearest < R).ravel(), farthest


def test_cylinder_chords_model_the_cylinder():
    w = synth.workload("slice64")
    h = w.histories()
    R = 0.5 * w.diameter
    meets, farthest = _disk_masks(w.grid, R)
    hull = oracle.hull(w.grid, h, wepl_in=1.0, wepl_out=0.0, min_in=1, max_out=0)
    assert not np.any(hull.astype(bool) & ~meets)           # chords stay in the convex object
    inner = (farthest < R - 2.0 * w.grid.vx).ravel()
    assert np.all(hull.astype(bool)[inner])                 # and cover its interior
    cin, _ = oracle.hull_counts(w.grid, h, 1.0, 0.0)
    assert np.array_equal(hull, (cin >= 1).astype(np.uint8))
    k = int(cin[cin > 0].min()) + 1                         # drops the least-crossed voxels
    strict = oracle.hull(w.grid, h, wepl_in=1.0, wepl_out=0.0, min_in=k, max_out=0)
    assert np.all(strict <= hull) and strict.sum() < hull.sum()
    assert np.array_equal(strict, (cin >= k).astype(np.uint8))


def test_missing_lines_carve_only_outside():
    w = synth.workload("slice64")
    g = w.grid
    R = 0.5 * w.diameter
    rng = np.random.default_rng(9)
    n = 3000
    phi = rng.uniform(0, 2 * math.pi, n)
    t = rng.uniform(R + 0.5, 45.0 * math.sqrt(2.0), n) * rng.choice([-1.0, 1.0], n)
    u = np.stack([np.cos(phi), np.sin(phi)], 1)
    v = np.stack([-np.sin(phi), np.cos(phi)], 1)
    c = t[:, None] * v
    p0 = np.concatenate([c - 70.0 * u, np.zeros((n, 1))], 1)
    p1 = np.concatenate([c + 70.0 * u, np.zeros((n, 1))], 1)
    miss = lines(p0, p1, rng.normal(0.0, 0.3, n))
    meets, farthest = _disk_masks(g, R)
    _, cout = oracle.hull_counts(g, miss, 1.0, 1.0)
    assert cout.sum() > 0 and not np.any((cout > 0) & (farthest < R).ravel())
    h = w.histories()
    both = {k: np.concatenate([h[k], miss[k]]) for k in h}
    hull = oracle.hull(g, both, wepl_in=1.0, wepl_out=1.0, min_in=1, max_out=0)
    sm = oracle.hull(g, h, wepl_in=1.0, wepl_out=1.0, min_in=1, max_out=0)
    assert np.all(hull <= sm)
    assert np.array_equal(hull.astype(bool), sm.astype(bool) & (cout == 0))
