"""Serving on the GPU: requests of different grids, history counts and
parameters run concurrently on their own contexts; each result must equal
the same request run alone (within 1e-5 relative: only the order of float
atomics differs) and, for requests of two grids, the oracle (1e-4), and a
failing request must fail alone."""
import numpy as np
import pytest

import oracle
from paper_1803_01112_amd import synth, tvs

pytestmark = pytest.mark.gpu


def rel_err(x, ref):
    ref = np.asarray(ref, np.float64)
    return float(np.max(np.abs(np.asarray(x, np.float64) - ref) / np.maximum(np.abs(ref), 0.1)))


def requests():
    out = []
    specs = [("vol64", 60_000, 1e-4, 3, 0.75, 4), ("vol64", 150_000, 2e-4, 1, 0.5, 3),
             ("vol128", 120_000, 1.5e-4, 5, 0.85, 3), ("slice64", 40_000, 0.05, 2, 0.95, 4),
             ("vol64", 20_000, 1e-4, 6, 0.65, 5), ("vol128", 60_000, 2e-4, 4, 0.75, 2)]
    for q, (name, n, lam, N, alpha, K) in enumerate(specs):
        w = synth.workload(name, n_hist=n)
        out.append(dict(w=w, h=w.histories(), lam=lam, N=N, alpha=alpha, K=K, seed=77 + q,
                        x0=w.initial_image()))
    return out


def test_mix_equals_alone():
    reqs = requests()
    alone = []
    for r in reqs:
        with tvs.Context(r["w"].grid, block_size=3200, chunk_histories=65536) as ctx:
            ctx.load_histories(r["h"])
            ctx.set_image(r["x0"])
            ctx.iterate(r["K"], r["lam"], r["N"], r["alpha"], seed=r["seed"])
            alone.append(ctx.get_image())
    with tvs.Server(max_active=3, chunk_histories=65536) as s:
        ids = [s.submit(r["w"].grid, r["h"], lam=r["lam"], N=r["N"], alpha=r["alpha"],
                        K=r["K"], seed=r["seed"], x0=r["x0"]) for r in reqs]
        res = [s.wait(i) for i in ids]
        c = s.counters()
    assert c["completed"] == len(reqs) and c["failed"] == 0
    assert c["peak_bytes"] <= c["budget_bytes"]
    assert c["peak_active"] >= 2          # requests really overlapped
    for q, ((img, info), ref) in enumerate(zip(res, alone)):
        assert info["status"] == 0, q
        assert rel_err(img, ref) <= 1e-5, q
    # two requests of the mix, of different grids, against the oracle
    for q in (1, 2):
        r = reqs[q]
        rows = oracle.build_rows(r["w"].grid, r["h"], 1.0)
        S = oracle.Superiorizer(r["w"].grid, rows, r["x0"], 3200)
        S.iterate(r["K"], r["lam"], r["N"], r["alpha"], seed=r["seed"])
        e = rel_err(res[q][0], S.x)
        print(f"served request {q} ({r['w'].name}, {len(r['h']['ex'])} histories): "
              f"vs oracle {e:.2e}")
        assert e <= 1e-4, q


def test_failing_request_fails_alone():
    reqs = requests()[:3]
    bad = {k: v.copy() for k, v in reqs[1]["h"].items()}
    bad["wepl"][5] = np.inf
    with tvs.Server(max_active=2, chunk_histories=65536) as s:
        a = s.submit(reqs[0]["w"].grid, reqs[0]["h"], lam=1e-4, N=1, alpha=0.5, K=1)
        b = s.submit(reqs[1]["w"].grid, bad, lam=1e-4, N=1, alpha=0.5, K=1)
        c = s.submit(reqs[2]["w"].grid, reqs[2]["h"], lam=1e-4, N=1, alpha=0.5, K=1)
        ra, rb, rc = s.wait(a), s.wait(b), s.wait(c)
    assert ra[1]["status"] == 0 and rc[1]["status"] == 0
    assert rb[0] is None and rb[1]["status"] == tvs.TVS_EINVAL
