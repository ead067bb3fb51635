"""Autotuning of the launch shape: the tuner must leave the image as it was,
pick one of its measured candidates (on the fly also the share of row chunks
formed at full occupancy), reuse a cached choice, and the tuned context must
still match the oracle."""
import os

import numpy as np
import pytest

import oracle
from paper_1803_01112_amd import synth, tvs

pytestmark = pytest.mark.gpu


def rel_err(x, ref):
    return float(np.max(np.abs(np.asarray(x, np.float64) - ref) / np.maximum(np.abs(ref), 0.1)))


@pytest.mark.parametrize("path_mode", ["otf", "f32"])
def test_autotune_keeps_image_and_parity(tmp_path, path_mode):
    w = synth.workload("slice64", n_hist=30_000)
    h = w.histories()
    x0 = w.initial_image()
    cache = os.path.join(tmp_path, "tune.txt")
    with tvs.Context(w.grid, block_size=64, mlp_step_mm=2.0, path_mode=path_mode,
                     chunk_histories=6400) as ctx:
        ctx.load_histories(h)
        ctx.set_image(x0)
        r = ctx.autotune(0.05, cache)
        assert not r["from_cache"] and r["candidates"]
        assert (r["tile_threads"], r["sweep_kernel"]) in {(c["threads"], c["sweep"])
                                                           for c in r["candidates"]}
        np.testing.assert_array_equal(ctx.get_image(), x0)
        if path_mode == "otf":
            # whole sweeps for the share of full-occupancy row chunks (5 chunks here)
            assert [c["pct"] for c in r["fill_candidates"]] == [0, 20, 40, 60, 80, 100]
            assert all(c["ms"] > 0 for c in r["fill_candidates"])
            assert r["fill_wide_pct"] == min(r["fill_candidates"], key=lambda c: c["ms"])["pct"]
            np.testing.assert_array_equal(ctx.get_image(), x0)
        else:
            assert r["fill_candidates"] == []
        r2 = ctx.autotune(0.05, cache)
        assert r2["from_cache"] and r2["tile_threads"] == r["tile_threads"]
        assert r2["fill_wide_pct"] == r["fill_wide_pct"]
        ctx.iterate(2, 0.05, 3, 0.75, seed=5)
        x = ctx.get_image()
    rows = oracle.build_rows(w.grid, h, 2.0)
    S = oracle.Superiorizer(w.grid, rows, x0, 64)
    S.iterate(2, 0.05, 3, 0.75, seed=5)
    assert rel_err(x, S.x) <= 1e-4
