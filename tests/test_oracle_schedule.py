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


# ---------------------------------------------------------------------------
# The retry branch of the checked step and the length of the unchecked step,
# pinned against images stepped explicitly here.  TV is recomputed with numpy
# (per-slice forward differences, Section IV's definition of TV);
# the direction v = -grad/||grad|| takes the oracle's subgradient, which
# tests/test_oracle_tv.py pins against finite differences.
# ---------------------------------------------------------------------------
def _empty_rows():
    return dict(row_off=np.zeros(1, np.int64), idx=np.zeros(0, np.int32),
                chord=np.zeros(0), norm2=np.zeros(0), wepl=np.zeros(0))


def _np_tv(grid, x):
    v = np.asarray(x, np.float64).reshape(grid.nz, grid.ny, grid.nx)
    dx = np.zeros_like(v)
    dy = np.zeros_like(v)
    dx[:, :, :-1] = v[:, :, 1:] - v[:, :, :-1]
    dy[:, :-1, :] = v[:, 1:, :] - v[:, :-1, :]
    return float(np.sum(np.sqrt(dx * dx + dy * dy)))


def _v(grid, x):
    """v = -grad phi / ||grad phi|| from the oracle's subgradient."""
    g, n2 = oracle.tv_grad(grid, x)
    gn = np.sqrt(n2)
    return -g / gn if gn > 0 else np.zeros_like(g)


def test_checked_step_retries_with_beta_recomputed():
    """Appendix C, checked NTVS (reading: beta = alpha^ell recomputed after
    every ell += 1).  A small-amplitude image and alpha = 1/2 make the first
    tries (beta = 1, 1/2, ...) overshoot, so the step needs several tries:
    every rejected try t must raise TV, the accepted image must be
    x + alpha^(ell0 + tries - 1) v with TV not above TV(x), and ell must
    advance by exactly the number of tries.  The literal listing (beta never
    updated inside the loop) rejects forever and fails here."""
    g = synth.Grid(16, 16, 1, 1.0, 1.0, 1.0, -8.0, -8.0, -0.5)
    rng = np.random.default_rng(31)
    x0 = 0.01 * rng.standard_normal(g.nvox)
    alpha = 0.5
    S = oracle.Superiorizer(g, _empty_rows(), x0, 10)
    recs = S.iterate(1, 1e-3, 1, alpha, tv_check=1, seed=4, max_tries=200)
    r = recs[0]
    tries, ell0 = r["tries"], r["ell_start"]
    assert ell0 == S.ell_log[0] == 0              # rand(0, 0) = 0
    assert r["accepted"] == 1 and tries >= 3
    v = _v(g, x0)
    phx = _np_tv(g, x0)
    assert r["phi_x"] == pytest.approx(phx, rel=1e-13)
    for t in range(1, tries):                     # every rejected try raised TV
        z = x0 + alpha ** (ell0 + t - 1) * v
        assert _np_tv(g, z) > phx
    z = x0 + alpha ** (ell0 + tries - 1) * v      # the accepted try
    np.testing.assert_allclose(S.x, z, rtol=0, atol=1e-15)
    assert _np_tv(g, S.x) <= phx
    assert r["phi_z"] == pytest.approx(_np_tv(g, S.x), rel=1e-13)
    assert S.state.ell == ell0 + tries


def test_checked_steps_chain_ell_across_steps_and_cycles():
    """Several checked steps and cycles: each step starts at the ell its
    predecessor left (start + tries), each cycle draws ell_k = rand(k, ell)
    from the pinned SplitMix64 stream, and every step's image is the one
    stepped here with beta = alpha^(start + tries - 1)."""
    g = synth.Grid(12, 10, 2, 1.0, 1.0, 1.0, -6.0, -5.0, -1.0)
    rng = np.random.default_rng(5)
    x0 = 0.02 * rng.standard_normal(g.nvox)
    alpha, N, K, seed = 0.6, 3, 3, 123
    S = oracle.Superiorizer(g, _empty_rows(), x0, 10)
    x = x0.copy()
    state, ell = seed, 0
    for k in range(K):
        recs = S.iterate(1, 1e-3, N, alpha, tv_check=1, seed=seed, max_tries=500)
        ell, state = oracle.rand_ell(k, ell, state)
        assert S.ell_log[k] == ell
        for r in recs:
            assert r["ell_start"] == ell and r["accepted"] == 1
            v = _v(g, x)
            phx = _np_tv(g, x)
            for t in range(1, r["tries"]):
                assert _np_tv(g, x + alpha ** (ell + t - 1) * v) > phx
            x = x + alpha ** (ell + r["tries"] - 1) * v
            assert _np_tv(g, x) <= phx
            ell += r["tries"]
        np.testing.assert_allclose(S.x, x, rtol=0, atol=1e-14)
        assert S.state.ell == ell
    assert any(r["tries"] > 1 for r in S.steps)


def test_checked_step_gives_up_after_max_tries():
    """A bounded retry loop leaves the image unchanged and logs the step as
    not accepted when no try within max_tries lowers TV."""
    g = synth.Grid(16, 16, 1, 1.0, 1.0, 1.0, -8.0, -8.0, -0.5)
    rng = np.random.default_rng(31)
    x0 = 0.01 * rng.standard_normal(g.nvox)
    S = oracle.Superiorizer(g, _empty_rows(), x0, 10)
    recs = S.iterate(1, 1e-3, 1, 0.5, tv_check=1, seed=4, max_tries=1)
    assert recs[0]["tries"] == 1 and recs[0]["accepted"] == 0
    np.testing.assert_array_equal(S.x, x0)
    assert S.state.ell == 1


def test_unchecked_ntvs_step_length_is_alpha_to_ell():
    """Appendix C without the check: step n of cycle k moves the image by
    exactly alpha^(ell_k + n) along v, with ell_k = rand(k, ell) drawn once
    per cycle; the image is followed step by step here (empty system, so
    P_T is the identity)."""
    g = synth.Grid(12, 12, 1, 1.0, 1.0, 1.0, -6.0, -6.0, -0.5)
    rng = np.random.default_rng(77)
    x0 = rng.standard_normal(g.nvox)
    alpha, N, K, seed = 0.75, 3, 5, 2024
    S = oracle.Superiorizer(g, _empty_rows(), x0, 10)
    x = x0.copy()
    state, ell = seed, 0
    for k in range(K):
        prev = S.x.copy()
        S.iterate(1, 1e-3, N, alpha, seed=seed)
        ell, state = oracle.rand_ell(k, ell, state)
        assert S.ell_log[k] == ell
        for n in range(N):
            step = alpha ** ell * _v(g, x)
            assert np.linalg.norm(step) == pytest.approx(alpha ** ell, rel=1e-13)
            x = x + step
            ell += 1
        np.testing.assert_allclose(S.x, x, rtol=0, atol=1e-13)
        if N == 1:
            assert np.linalg.norm(S.x - prev) == pytest.approx(alpha ** S.ell_log[k], rel=1e-12)
    assert S.state.ell == ell
    # a draw below the previous end happened (the schedule is not the N = 1 one)
    assert any(S.ell_log[k] < S.ell_log[k - 1] + N for k in range(1, K))


def test_unchecked_single_step_length():
    """N = 1: the cycle's one step has length alpha^(ell_k) exactly."""
    g = synth.Grid(10, 10, 1, 1.0, 1.0, 1.0, -5.0, -5.0, -0.5)
    x0 = np.random.default_rng(3).standard_normal(g.nvox)
    S = oracle.Superiorizer(g, _empty_rows(), x0, 10)
    for k in range(4):
        prev = S.x.copy()
        S.iterate(1, 1e-3, 1, 0.8, seed=9)
        assert np.linalg.norm(S.x - prev) == pytest.approx(0.8 ** S.ell_log[k], rel=1e-12)
