"""GPU parity of the TV-reduction check decided on the device (Appendix C's
checked NTVS with beta = alpha^ell recomputed after every ell += 1, and
Appendix B's OTVS): one launch tries 16 step lengths at once, the last
workgroup decides and, when none passes, tries further rounds alone.

The oracle replays the GPU's number of tries per step and reports where its
own float64 decision would differ; such a difference is allowed only where
TV(z) and TV(x) agree to within 1e-6 relative, the agreement of the two
sides' TV values (both sum float64 terms, in different orders, of images
whose DROP updates were summed differently: exact fixed point on the GPU,
float64 in row order in the oracle; the images drift apart over the
cycles by far less than their 1e-4 tolerance).  Images: 1e-4 relative RSP
(floor 0.1).
"""
import numpy as np
import pytest

import oracle
from paper_1803_01112_amd import synth, tvs

pytestmark = pytest.mark.gpu
TOL = 1e-4


def rel_err(x, ref):
    ref = np.asarray(ref, np.float64)
    return float(np.max(np.abs(np.asarray(x, np.float64) - ref) / np.maximum(np.abs(ref), 0.1)))


@pytest.fixture(scope="module")
def few():
    """The slice grid with a handful of histories: DROP barely moves the
    image, so the TV steps decide it."""
    w = synth.workload("slice64", n_hist=40)
    h = w.histories()
    rows = oracle.build_rows(w.grid, h, 2.0)
    return w, h, rows


def check_replay(log, recs):
    for r, g in zip(recs, log):
        assert g["ell_start"] == r["ell_start"]
        if r["disagree"]:
            assert r["worst_margin"] <= 1e-6 * r["phi_x"]
        assert g["phi_x"] == pytest.approx(r["phi_x"], rel=1e-6)
        if g["accepted"]:
            assert g["phi_z"] == pytest.approx(r["phi_z"], rel=1e-6)


def run_gpu(w, h, x0, calls, max_tries=0):
    with tvs.Context(w.grid, block_size=64, mlp_step_mm=2.0, max_tries=max_tries) as ctx:
        ctx.load_histories(h)
        ctx.set_image(x0)
        for kw in calls:
            ctx.iterate(**kw)
        x = ctx.get_image()
        log = ctx.step_log()
        st = ctx.stats()
    return x, log, st


def test_many_tries_need_further_rounds(few):
    """A small-amplitude image (noise of 3e-4 on 1.0) and alpha = 0.95:
    unit-length steps overshoot, and the first accepted try of some steps
    lies well past the first 16 (the oracle's own run takes 71, 19 and 57)."""
    w, h, rows = few
    rng = np.random.default_rng(12)
    x0 = (1.0 + 3e-4 * rng.standard_normal(w.grid.nvox)).astype(np.float32)
    call = dict(K=3, lam=1e-4, N=2, alpha=0.95, tv_check=True, seed=5)
    x, log, st = run_gpu(w, h, x0, [call])
    print("tries per step:", [r["tries"] for r in log])
    assert max(r["tries"] for r in log) > 16
    assert all(r["accepted"] for r in log)
    S = oracle.Superiorizer(w.grid, rows, x0, 64)
    recs = S.iterate(3, 1e-4, 2, 0.95, tv_check=1, seed=5,
                     replay_tries=[r["tries"] for r in log])
    check_replay(log, recs)
    assert st["ell"] == S.state.ell
    assert st["tries"] == sum(r["tries"] for r in log)
    assert rel_err(x, S.x) <= TOL


def test_steps_give_up_after_max_tries(few):
    """With max_tries = 3 a step whose first three tries all raise TV gives
    up: image unchanged by it, ell advanced by 3, logged as not accepted;
    the GPU's records equal the oracle's own."""
    w, h, rows = few
    rng = np.random.default_rng(12)
    x0 = (1.0 + 3e-4 * rng.standard_normal(w.grid.nvox)).astype(np.float32)
    call = dict(K=2, lam=1e-4, N=2, alpha=0.95, tv_check=True, seed=5)
    x, log, st = run_gpu(w, h, x0, [call], max_tries=3)
    S = oracle.Superiorizer(w.grid, rows, x0, 64)
    recs = S.iterate(2, 1e-4, 2, 0.95, tv_check=1, seed=5, max_tries=3)
    print("gpu:", [(r["tries"], r["accepted"]) for r in log])
    assert any(not r["accepted"] for r in log)
    assert all(r["tries"] <= 3 for r in log)
    assert [(r["tries"], r["accepted"]) for r in log] == \
        [(r["tries"], r["accepted"]) for r in recs]
    assert st["ell"] == S.state.ell
    assert rel_err(x, S.x) <= TOL


def test_checked_and_unchecked_calls_interleaved(few):
    """The schedule moves between the device (checked calls) and the host
    (unchecked calls) without losing ell or the RNG stream."""
    w, h, rows = few
    rng = np.random.default_rng(3)
    x0 = (1.0 + 0.05 * rng.standard_normal(w.grid.nvox)).astype(np.float32)
    calls = [dict(K=2, lam=0.02, N=3, alpha=0.8, tv_check=True, seed=11),
             dict(K=2, lam=0.02, N=3, alpha=0.8, tv_check=False, seed=11),
             dict(K=1, lam=0.02, N=3, alpha=0.8, tv_check=True, seed=11),
             dict(K=2, lam=0.02, N=3, alpha=0.8, tv_check=True, seed=11)]
    x, log, st = run_gpu(w, h, x0, calls)
    S = oracle.Superiorizer(w.grid, rows, x0, 64)
    done = 0
    for c in calls:
        n = c["K"] * c["N"]
        S.iterate(c["K"], c["lam"], c["N"], c["alpha"], tv_check=int(c["tv_check"]),
                  seed=c["seed"], replay_tries=[r["tries"] for r in log[done:done + n]]
                  if c["tv_check"] else None)
        done += n
    assert len(log) == done
    check_replay(log, S.steps)
    assert st["ell"] == S.state.ell and st["k"] == 7
    assert rel_err(x, S.x) <= TOL


def test_step_records_beyond_the_device_buffer(few):
    """More checked steps in one call than the device holds records for
    (4096): the records are copied back part way; the log, ell and image
    equal those of the same 700 cycles run as seven calls of 100 (the GPU
    path is deterministic: exact integer DROP sums, fixed-order TV sums)."""
    w, h, rows = few
    rng = np.random.default_rng(4)
    x0 = (1.0 + 0.05 * rng.standard_normal(w.grid.nvox)).astype(np.float32)
    call = dict(K=700, lam=1e-3, N=6, alpha=0.7, tv_check=True, seed=8)
    xa, la, sa = run_gpu(w, h, x0, [call])
    xb, lb, sb = run_gpu(w, h, x0, [dict(call, K=100)] * 7)
    assert len(la) == 4200 and sa["steps"] == 4200
    assert [r["k"] for r in la[::6]] == list(range(700))
    assert la == lb
    assert sa["ell"] == sb["ell"] and sa["tries"] == sb["tries"] == sum(r["tries"] for r in la)
    np.testing.assert_array_equal(xa, xb)
