"""Scheduling policy of the serving layer, on the CPU (simulated executor: a
request sleeps in proportion to its history-cycles instead of running).

Checked: first-in first-out admission, the HBM budget is never exceeded,
a request too large for the budget is refused at submit, requests that
arrive while others run are admitted as slots free (continuous batching),
and shutdown fails only what never started.
"""
import time

import numpy as np
import pytest

from paper_1803_01112_amd import synth, tvs

GRID = synth.centered_grid(16, 16, 2, 1.0, 1.0, 2.5)


def fake_hist(n):
    return {k: np.zeros(n, np.float32) for k in synth.HIST_FIELDS}


@pytest.fixture
def server():
    s = tvs.Server(simulate=True, max_active=3, hbm_budget_bytes=1 << 30,
                   sim_ns_per_history_cycle=50.0)
    yield s
    s.close()


def test_fifo_admission_and_completion(server):
    ids = [server.submit(GRID, fake_hist(2000 * (q + 1)), lam=1e-4, N=1, alpha=0.5, K=2)
           for q in range(8)]
    infos = [server.wait(r)[1] for r in ids]
    assert [i["admit_order"] for i in infos] == list(range(1, 9))
    assert all(i["state"] == 2 and i["status"] == 0 for i in infos)
    c = server.counters()
    assert c["completed"] == 8 and c["failed"] == 0
    assert c["peak_active"] <= 3
    assert c["in_use_bytes"] == 0


def test_budget_never_exceeded_and_head_blocks():
    one = None
    with tvs.Server(simulate=True, max_active=8, hbm_budget_bytes=1 << 40,
                    sim_ns_per_history_cycle=1.0) as probe:
        one = probe.footprint(GRID, fake_hist(100_000))
    budget = int(2.5 * one)            # room for two such requests at a time
    with tvs.Server(simulate=True, max_active=8, hbm_budget_bytes=budget,
                    sim_ns_per_history_cycle=200.0) as s:
        ids = [s.submit(GRID, fake_hist(100_000), lam=1e-4, N=1, alpha=0.5, K=1)
               for _ in range(6)]
        for r in ids:
            img, info = s.wait(r)
            assert info["status"] == 0
        c = s.counters()
        assert c["peak_bytes"] <= budget
        assert c["peak_active"] == 2


def test_oversized_request_refused(server):
    with pytest.raises(tvs.TvsError) as e:
        server.submit(GRID, fake_hist(30_000_000), lam=1e-4, N=1, alpha=0.5, K=1)
    assert e.value.status == tvs.TVS_ENOMEM


def test_invalid_request_refused(server):
    bad = synth.Grid(0, 16, 2, 1.0, 1.0, 2.5, 0, 0, 0)
    with pytest.raises(tvs.TvsError) as e:
        server.submit(bad, fake_hist(10), lam=1e-4, N=1, alpha=0.5, K=1)
    assert e.value.status == tvs.TVS_EINVAL


def test_continuous_admission_overlaps_arrivals(server):
    first = [server.submit(GRID, fake_hist(200_000), lam=1e-4, N=1, alpha=0.5, K=1)
             for _ in range(3)]
    time.sleep(0.002)
    late = server.submit(GRID, fake_hist(1000), lam=1e-4, N=1, alpha=0.5, K=1)
    _, info_late = server.wait(late)
    infos = [server.wait(r)[1] for r in first]
    # the late request waited for a slot, then started before all early ones ended
    assert info_late["admit_ms"] >= min(i["done_ms"] for i in infos) - 1e-6
    assert info_late["done_ms"] <= max(i["done_ms"] for i in infos) + 50.0


def test_shutdown_cancels_only_queued():
    s = tvs.Server(simulate=True, max_active=1, hbm_budget_bytes=1 << 30,
                   sim_ns_per_history_cycle=1000.0)
    a = s.submit(GRID, fake_hist(20_000), lam=1e-4, N=1, alpha=0.5, K=1)
    b = s.submit(GRID, fake_hist(20_000), lam=1e-4, N=1, alpha=0.5, K=1)
    time.sleep(0.005)
    ia = s.query(a)
    s.close()
    assert ia["state"] in (1, 2)


@pytest.mark.parametrize("name,n", [("slice64", 20_000), ("vol64", 50_000), ("vol200", 30_000),
                                    ("vol256", 20_000)])
def test_store_estimate_bounds_the_rows(name, n):
    """The admission estimate of a path store comes from the histories'
    straight entry-exit lines with a margin for the most likely path's bend;
    it must hold every row entry the oracle forms for those histories (the
    float32 and 6-byte stores differ by 2 bytes per estimated entry), and
    stay well below the grid-wide bound it replaced."""
    import oracle
    w = synth.workload(name, n_hist=n)
    h = w.histories()
    nnz = len(oracle.build_rows(w.grid, h, min(w.grid.vx, w.grid.vy))["idx"])
    with tvs.Server(simulate=True, max_active=1, hbm_budget_bytes=1 << 50,
                    sim_ns_per_history_cycle=1.0) as s:
        f32 = s.footprint(w.grid, h, path_mode="f32")
        q16 = s.footprint(w.grid, h, path_mode="q16")
    est = (f32 - q16) / 2.0
    assert nnz <= est <= 2.5 * nnz, (nnz, est)
    span = (w.grid.nx * w.grid.vx + w.grid.ny * w.grid.vy) / min(w.grid.vx, w.grid.vy)
    grid_wide = n * (int(0.8 * span) + w.grid.nz + 8)
    assert est < grid_wide
