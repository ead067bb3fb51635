"""Pins of the oracle's voxel walk (row formation).

Each history's equation holds the chord lengths of its path through the
voxels (arXiv 1803.01112, Section I); the paper does not say how they are
computed.  The oracle walks every polyline segment with Siddon's parametric
method and assigns each piece to the voxel containing its midpoint.  Pinned
here by: total chord = in-box polyline length (clipping written
independently, Liang-Barsky), brute-force supersampled voxel membership on
tiny grids, exact voxel-width chords for axis-aligned rays through voxel
centres, and structural invariants (no empty or repeated consecutive entry).
"""
import numpy as np
import pytest

import oracle
from paper_1803_01112_amd.synth import Grid


def clipped_length(grid, p, q):
    """Length of segment p->q inside the grid box (Liang-Barsky clipping)."""
    lo = np.array([grid.ox, grid.oy, grid.oz])
    hi = lo + np.array([grid.nx * grid.vx, grid.ny * grid.vy, grid.nz * grid.vz])
    d = q - p
    t0, t1 = 0.0, 1.0
    for a in range(3):
        if d[a] == 0.0:
            if p[a] < lo[a] or p[a] > hi[a]:
                return 0.0
            continue
        ta, tb = (lo[a] - p[a]) / d[a], (hi[a] - p[a]) / d[a]
        ta, tb = min(ta, tb), max(ta, tb)
        t0, t1 = max(t0, ta), min(t1, tb)
    return max(0.0, t1 - t0) * float(np.linalg.norm(d))


GRIDS = [Grid(4, 4, 2, 1.0, 1.0, 2.5, -2.0, -2.0, -2.5),
         Grid(7, 5, 3, 0.7, 1.3, 0.9, -2.1, -3.0, -1.0),
         Grid(16, 16, 1, 2.0, 2.0, 2.0, -16.0, -16.0, -1.0)]


@pytest.mark.parametrize("grid", GRIDS)
def test_total_chord_equals_inbox_length(grid):
    rng = np.random.default_rng(1)
    ext = np.array([grid.nx * grid.vx, grid.ny * grid.vy, grid.nz * grid.vz])
    lo = np.array([grid.ox, grid.oy, grid.oz])
    for _ in range(200):
        n = rng.integers(2, 8)
        pts = lo + rng.uniform(-0.3, 1.3, size=(n, 3)) * ext
        idx, ch, n2 = oracle.walk_polyline(grid, pts)
        want = sum(clipped_length(grid, pts[s], pts[s + 1]) for s in range(n - 1))
        assert ch.sum() == pytest.approx(want, rel=1e-12, abs=1e-12)
        assert n2 == pytest.approx(float((ch ** 2).sum()), rel=1e-14)
        assert np.all(ch > 0)
        assert np.all(idx[1:] != idx[:-1])
        assert np.all((idx >= 0) & (idx < grid.nvox))


def supersample(grid, p, q, n=400_000):
    """Voxel run-lengths along p->q by dense midpoint sampling."""
    t = (np.arange(n) + 0.5) / n
    pts = p[None, :] + t[:, None] * (q - p)[None, :]
    g = (pts - [grid.ox, grid.oy, grid.oz]) / [grid.vx, grid.vy, grid.vz]
    c = np.floor(g).astype(np.int64)
    inside = np.all((c >= 0) & (c < [grid.nx, grid.ny, grid.nz]), axis=1)
    lin = np.where(inside, c[:, 0] + grid.nx * (c[:, 1] + grid.ny * c[:, 2]), -1)
    seglen = float(np.linalg.norm(q - p)) / n
    runs = []
    for v in lin:
        if runs and runs[-1][0] == v:
            runs[-1][1] += seglen
        else:
            runs.append([v, seglen])
    return [(v, l) for v, l in runs if v >= 0]


def test_bruteforce_membership_tiny_grid():
    grid = GRIDS[0]
    rng = np.random.default_rng(2)
    for _ in range(25):
        p = rng.uniform([-2.5, -2.5, -3.0], [2.5, 2.5, 3.0])
        q = rng.uniform([-2.5, -2.5, -3.0], [2.5, 2.5, 3.0])
        idx, ch, _ = oracle.walk_polyline(grid, np.array([p, q]))
        runs = supersample(grid, p, q)
        # pieces shorter than a few samples may be missed by sampling
        tiny = 4 * float(np.linalg.norm(q - p)) / 400_000
        mine = [(int(v), float(l)) for v, l in zip(idx, ch) if l > tiny]
        ref = [(int(v), float(l)) for v, l in runs if l > tiny]
        assert [v for v, _ in mine] == [v for v, _ in ref]
        for (_, a), (_, b) in zip(mine, ref):
            assert a == pytest.approx(b, abs=3 * tiny)


def test_axis_aligned_ray_through_centres():
    grid = Grid(10, 8, 3, 1.5, 2.0, 2.5, -7.5, -8.0, -3.75)
    for iy in range(grid.ny):
        for iz in range(grid.nz):
            y = grid.oy + (iy + 0.5) * grid.vy
            z = grid.oz + (iz + 0.5) * grid.vz
            pts = np.array([[-20.0, y, z], [20.0, y, z]])
            idx, ch, _ = oracle.walk_polyline(grid, pts)
            want = np.arange(grid.nx) + grid.nx * (iy + grid.ny * iz)
            np.testing.assert_array_equal(idx, want)
            np.testing.assert_allclose(ch, grid.vx, rtol=1e-13)


def test_ray_on_plane_goes_to_higher_voxel():
    grid = Grid(4, 4, 1, 1.0, 1.0, 1.0, 0.0, 0.0, -0.5)
    idx, ch, _ = oracle.walk_polyline(grid, np.array([[-1.0, 2.0, 0.0], [5.0, 2.0, 0.0]]))
    np.testing.assert_array_equal(idx, np.arange(4) + 4 * 2)
    np.testing.assert_allclose(ch, 1.0)


def test_vertex_inside_voxel_merges_entry():
    grid = Grid(4, 4, 1, 1.0, 1.0, 1.0, 0.0, 0.0, -0.5)
    pts = np.array([[0.2, 0.5, 0.0], [0.6, 0.55, 0.0], [3.5, 0.6, 0.0]])
    idx, ch, _ = oracle.walk_polyline(grid, pts)
    np.testing.assert_array_equal(idx, [0, 1, 2, 3])
    assert ch.sum() == pytest.approx(np.linalg.norm(pts[1] - pts[0]) +
                                     np.linalg.norm(pts[2] - pts[1]), rel=1e-14)


def test_reentry_is_a_separate_entry():
    grid = Grid(4, 4, 1, 1.0, 1.0, 1.0, 0.0, 0.0, -0.5)
    pts = np.array([[0.5, 0.5, 0.0], [1.5, 0.5, 0.0], [0.5, 0.6, 0.0]])
    idx, ch, n2 = oracle.walk_polyline(grid, pts)
    np.testing.assert_array_equal(idx, [0, 1, 0])
    assert n2 == pytest.approx(float((ch ** 2).sum()))


def test_rows_of_many_histories_consistent_with_single_walks():
    from paper_1803_01112_amd import synth
    w = synth.workload("slice64", n_hist=900)
    h = w.histories()
    rows = oracle.build_rows(w.grid, h, 2.0)
    for i in (0, 17, 450, 899):
        hh = [float(h[k][i]) for k in synth.HIST_FIELDS[:12]]
        pts = oracle.mlp_polyline(hh, 2.0)
        idx, ch, n2 = oracle.walk_polyline(w.grid, pts)
        a, b = rows["row_off"][i], rows["row_off"][i + 1]
        np.testing.assert_array_equal(rows["idx"][a:b], idx)
        np.testing.assert_array_equal(rows["chord"][a:b], ch)
        assert rows["norm2"][i] == n2
