"""Pins of the oracle's schedule and superiorization driver.

NTVS (arXiv 1803.01112, Appendix C): ell_k = rand(k, ell_{k-1}) once per
cycle, N steps with beta = alpha^ell and ell += 1 after each, then P_T.
Section III-B states the invariants pinned here: with N = 1 and no check,
ell_{k-1} = k always (ell is never decreased), and k <= ell_k keeps
beta -> 0.  rand draws from SplitMix64, pinned against its published
reference outputs (tests/golden/splitmix64_state0.txt).  OTVS (Appendix B)
equals NTVS with the check, N = 1 and alpha = 1/2 whenever every first try
is accepted (Section III-B: alpha = 0.5 is the OTVS setting).
"""
import os

import numpy as np
import pytest

import oracle
from paper_1803_01112_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_state0.txt")


def test_splitmix64_reference_outputs():
    want = [int(l, 16) for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    got, _ = oracle.splitmix64(0, len(want))
    assert got == want


def test_rand_ell_range_and_uniformity():
    state = 99
    counts = np.zeros(7, int)
    for _ in range(70_000):
        r, state = oracle.rand_ell(3, 9, state)
        assert 3 <= r <= 9
        counts[r - 3] += 1
    chi2 = float(((counts - 10_000) ** 2 / 10_000).sum())
    assert chi2 < 30.0            # 6 dof: p ~ 4e-5
    r, _ = oracle.rand_ell(5, 5, 1)
    assert r == 5
    r, _ = oracle.rand_ell(6, 2, 1)   # ell below k: k
    assert r == 6


@pytest.fixture(scope="module")
def small_system():
    w = synth.workload("slice64", n_hist=6000)
    h = w.histories()
    rows = oracle.build_rows(w.grid, h, 2.0)
    return w, rows


def test_n1_without_check_never_decreases_ell(small_system):
    w, rows = small_system
    S = oracle.Superiorizer(w.grid, rows, w.initial_image(), 64)
    S.iterate(8, 1e-3, 1, 0.75, seed=5)
    assert S.ell_log == list(range(8))


@pytest.mark.parametrize("N", [2, 3, 6])
def test_ell_bounds(small_system, N):
    w, rows = small_system
    S = oracle.Superiorizer(w.grid, rows, w.initial_image(), 64)
    S.iterate(10, 1e-3, N, 0.75, seed=11)
    prev_end = 0
    for k, ell in enumerate(S.ell_log):
        assert k <= ell <= max(prev_end, k)
        prev_end = ell + N
    assert S.state.ell == S.ell_log[-1] + N


def test_seeded_runs_reproduce_and_resume(small_system):
    w, rows = small_system
    a = oracle.Superiorizer(w.grid, rows, w.initial_image(), 64)
    a.iterate(6, 1e-3, 3, 0.75, seed=42)
    b = oracle.Superiorizer(w.grid, rows, w.initial_image(), 64)
    b.iterate(2, 1e-3, 3, 0.75, seed=42)
    b.iterate(4, 1e-3, 3, 0.75, seed=42)
    np.testing.assert_array_equal(a.x, b.x)
    assert a.ell_log == b.ell_log


def test_n0_is_pure_drop(small_system):
    w, rows = small_system
    S = oracle.Superiorizer(w.grid, rows, w.initial_image(), 64)
    S.iterate(3, 0.05, 0, 0.75, seed=1)
    x = w.initial_image().astype(np.float64)
    for _ in range(3):
        oracle.drop_sweep(x, rows, 0.05, 64)
    np.testing.assert_array_equal(S.x, x)


def test_constant_image_check_accepts_first_try():
    g = synth.Grid(16, 16, 1, 1.0, 1.0, 1.0, -8.0, -8.0, -0.5)
    empty = dict(row_off=np.zeros(1, np.int64), idx=np.zeros(0, np.int32),
                 chord=np.zeros(0), norm2=np.zeros(0), wepl=np.zeros(0))
    S = oracle.Superiorizer(g, empty, np.full(g.nvox, 0.8), 10)
    recs = S.iterate(4, 1e-3, 3, 0.75, tv_check=1, seed=3)
    assert all(r["tries"] == 1 and r["accepted"] for r in recs)
    assert S.state.ell == S.ell_log[-1] + 3


def test_otvs_equals_checked_ntvs_when_first_tries_pass():
    g = synth.Grid(24, 24, 1, 1.0, 1.0, 1.0, -12.0, -12.0, -0.5)
    rng = np.random.default_rng(8)
    X, Y = np.meshgrid(np.arange(24), np.arange(24))
    x0 = (np.sin(X / 3.0) + np.cos(Y / 4.0)).ravel() * 5.0 + rng.normal(0, 0.01, 576)
    empty = dict(row_off=np.zeros(1, np.int64), idx=np.zeros(0, np.int32),
                 chord=np.zeros(0), norm2=np.zeros(0), wepl=np.zeros(0))
    a = oracle.Superiorizer(g, empty, x0, 10)
    ra = a.iterate(5, 1e-3, 1, 0.5, variant=1)
    b = oracle.Superiorizer(g, empty, x0, 10)
    rb = b.iterate(5, 1e-3, 1, 0.5, tv_check=1, variant=0, seed=77)
    assert all(r["tries"] == 1 for r in ra) and all(r["tries"] == 1 for r in rb)
    np.testing.assert_array_equal(a.x, b.x)
    assert b.ell_log == list(range(5))


def test_replay_of_own_decisions_agrees(small_system):
    w, rows = small_system
    a = oracle.Superiorizer(w.grid, rows, w.initial_image(), 64)
    ra = a.iterate(4, 0.02, 3, 0.9, tv_check=1, seed=9)
    assert any(r["tries"] > 1 for r in ra)
    b = oracle.Superiorizer(w.grid, rows, w.initial_image(), 64)
    rb = b.iterate(4, 0.02, 3, 0.9, tv_check=1, seed=9,
                   replay_tries=[r["tries"] for r in ra])
    assert all(r["disagree"] == 0 for r in rb)
    np.testing.assert_array_equal(a.x, b.x)


def test_decoupled_schedule_beta():
    """Section VI proposal: beta_{k,n} = alpha^n gamma^k; with an empty system
    and a single-voxel bump the first step moves the image by exactly beta."""
    g = synth.Grid(8, 8, 1, 1.0, 1.0, 1.0, -4.0, -4.0, -0.5)
    x0 = np.zeros(g.nvox)
    x0[27] = 1.0
    empty = dict(row_off=np.zeros(1, np.int64), idx=np.zeros(0, np.int32),
                 chord=np.zeros(0), norm2=np.zeros(0), wepl=np.zeros(0))
    S = oracle.Superiorizer(g, empty, x0, 10)
    S.iterate(1, 1e-3, 1, 0.6, variant=2, gamma=0.5)
    assert np.linalg.norm(S.x - x0) == pytest.approx(0.6, rel=1e-12)
    S2 = oracle.Superiorizer(g, empty, x0, 10)
    S2.iterate(2, 1e-3, 1, 0.6, variant=2, gamma=0.5)
    # second cycle (k = 1) steps by alpha * gamma
    step2 = np.linalg.norm(S2.x - S.x)
    assert step2 == pytest.approx(0.6 * 0.5, rel=1e-9)
