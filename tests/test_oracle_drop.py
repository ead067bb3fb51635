"""Pins of the oracle's feasibility sweep P_T (block-iterative DROP).

The paper runs DROP with blocks of 3200 or 25,600 histories (arXiv
1803.01112, Section III-D) and applies P_T once per cycle (Appendix C); it
prints no formula.  The oracle's reading: for each block, from one x,
r_i = (b_i - a_i.x)/||a_i||^2, c_j = sum r_i a_ij, s_j = number of entries
at j, x_j += lambda c_j/s_j.  Pinned here by mathematics: a single row
projection with lambda = 1 solves its own equation; on small consistent
full-column-rank systems the iteration converges to the unique solution
(dense least squares); a single block step is linear in lambda; voxels no
row touches never change.
"""
import numpy as np
import pytest

import oracle
from paper_1803_01112_amd.synth import Grid


def rows_from_lines(grid, lines):
    """CSR rows of straight lines through the grid, via the oracle's walk."""
    idx, ch, n2, off = [], [], [], [0]
    for p, q in lines:
        i, c, n = oracle.walk_polyline(grid, np.array([p, q]))
        idx.append(i)
        ch.append(c)
        n2.append(n)
        off.append(off[-1] + len(i))
    return dict(row_off=np.array(off, np.int64), idx=np.concatenate(idx).astype(np.int32),
                chord=np.concatenate(ch), norm2=np.array(n2))


def dense(rows, nvox):
    A = np.zeros((len(rows["norm2"]), nvox))
    for r in range(len(rows["norm2"])):
        a, b = rows["row_off"][r], rows["row_off"][r + 1]
        np.add.at(A[r], rows["idx"][a:b], rows["chord"][a:b])
    return A


def random_lines(rng, n, R=3.0):
    out = []
    for _ in range(n):
        phi = rng.uniform(0, 2 * np.pi)
        t = rng.uniform(-R * 0.9, R * 0.9)
        u = np.array([np.cos(phi), np.sin(phi)])
        tv = np.array([-u[1], u[0]])
        p = np.r_[-2 * R * u + t * tv, 0.0]
        q = np.r_[2 * R * u + t * tv, 0.0]
        out.append((p, q))
    return out


def test_single_row_projection_solves_its_equation():
    grid = Grid(8, 8, 1, 1.0, 1.0, 1.0, -4.0, -4.0, -0.5)
    rng = np.random.default_rng(0)
    for _ in range(20):
        rows = rows_from_lines(grid, random_lines(rng, 1, R=4.0))
        if rows["norm2"][0] == 0:
            continue
        assert len(np.unique(rows["idx"])) == len(rows["idx"])
        rows["wepl"] = np.array([rng.uniform(1, 10)])
        x = rng.uniform(0, 2, grid.nvox)
        oracle.drop_sweep(x, rows, 1.0, 1)
        A = dense(rows, grid.nvox)
        assert A[0] @ x == pytest.approx(rows["wepl"][0], rel=1e-14)


@pytest.mark.parametrize("B", [1, 5, 60])
def test_consistent_system_converges_to_unique_solution(B):
    grid = Grid(3, 3, 1, 2.0, 2.0, 2.0, -3.0, -3.0, -1.0)
    rng = np.random.default_rng(B)
    rows = rows_from_lines(grid, random_lines(rng, 60, R=3.0))
    keep = rows["norm2"] > 0
    assert keep.all()
    A = dense(rows, grid.nvox)
    assert np.linalg.matrix_rank(A) == grid.nvox
    xstar = rng.uniform(0.5, 1.5, grid.nvox)
    rows["wepl"] = A @ xstar
    sol = np.linalg.lstsq(A, rows["wepl"], rcond=None)[0]
    x = np.zeros(grid.nvox)
    for _ in range(3000):
        oracle.drop_sweep(x, rows, 1.0, B)
    np.testing.assert_allclose(x, sol, rtol=0, atol=1e-9)


def test_one_block_is_linear_in_lambda_and_leaves_untouched_voxels():
    grid = Grid(8, 8, 1, 1.0, 1.0, 1.0, -4.0, -4.0, -0.5)
    rng = np.random.default_rng(4)
    rows = rows_from_lines(grid, random_lines(rng, 12, R=2.5))
    rows["wepl"] = rng.uniform(1, 5, 12)
    x0 = rng.uniform(0, 2, grid.nvox)
    x1 = x0.copy()
    oracle.drop_sweep(x1, rows, 1.0, 12)
    xl = x0.copy()
    oracle.drop_sweep(xl, rows, 0.37, 12)
    np.testing.assert_allclose(xl - x0, 0.37 * (x1 - x0), rtol=1e-12, atol=1e-15)
    untouched = np.setdiff1d(np.arange(grid.nvox), rows["idx"])
    assert len(untouched) > 0
    np.testing.assert_array_equal(x1[untouched], x0[untouched])


def test_rows_without_entries_are_skipped():
    grid = Grid(4, 4, 1, 1.0, 1.0, 1.0, -2.0, -2.0, -0.5)
    lines = [(np.array([-5.0, 10.0, 0]), np.array([5.0, 10.0, 0]))]   # misses the grid
    rows = rows_from_lines(grid, lines)
    assert rows["norm2"][0] == 0
    rows["wepl"] = np.array([3.0])
    x = np.ones(grid.nvox)
    oracle.drop_sweep(x, rows, 1.0, 1)
    np.testing.assert_array_equal(x, 1.0)
