"""GPU parity of hull detection (tvs_hull_detect) against the oracle: space
modelling and space carving on every history's straight entry-exit line,
the voxels taken by the same midpoint walk as the rows, so the masks must
agree bit for bit (integer counts compared with integer thresholds).
Inputs: the phantom scans plus protons that pass beside the cylinder (their
WEPL only detector noise), in 2-D and 3-D, with and without carving, and
with the hull masking an initial iterate."""
import numpy as np
import pytest

import oracle
from paper_1803_01112_amd import synth, tvs

pytestmark = pytest.mark.gpu


def scan_with_misses(name, n_hist, n_miss, seed):
    w = synth.workload(name, n_hist=n_hist)
    h = w.histories()
    m = synth.miss_histories(w.grid, 0.5 * w.diameter, n_miss, seed)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n_hist + n_miss)
    return w, {k: np.concatenate([h[k], m[k]])[perm] for k in h}


@pytest.mark.parametrize("name,n_hist,n_miss", [("slice64", 60_000, 6_000),
                                                ("vol64", 300_000, 40_000)])
def test_hull_masks_match_the_oracle(name, n_hist, n_miss):
    w, h = scan_with_misses(name, n_hist, n_miss, 11)
    print(f"hull: {name}, {n_hist} + {n_miss} histories", flush=True)
    cases = [dict(wepl_in_mm=1.0, wepl_out_mm=0.0, min_in=1, max_out=0),
             dict(wepl_in_mm=1.0, wepl_out_mm=1.0, min_in=1, max_out=0),
             dict(wepl_in_mm=5.0, wepl_out_mm=1.0, min_in=20, max_out=2),
             dict(wepl_in_mm=-1e9, wepl_out_mm=1.0, min_in=0, max_out=0)]
    with tvs.Context(w.grid, block_size=3200) as ctx:
        ctx.load_histories(h)
        for c in cases:
            got = ctx.hull_detect(**c)
            want = oracle.hull(w.grid, h, wepl_in=c["wepl_in_mm"], wepl_out=c["wepl_out_mm"],
                               min_in=c["min_in"], max_out=c["max_out"])
            print(c, "inside", int(got.sum()), "of", got.size, flush=True)
            np.testing.assert_array_equal(got, want)
    carved = oracle.hull(w.grid, h, wepl_in=1.0, wepl_out=1.0, min_in=1, max_out=0)
    modelled = oracle.hull(w.grid, h, wepl_in=1.0, wepl_out=0.0, min_in=1, max_out=0)
    assert 0 < carved.sum() <= modelled.sum() < carved.size


def test_hull_masks_the_initial_iterate():
    w, h = scan_with_misses("vol64", 200_000, 30_000, 5)
    with tvs.Context(w.grid, block_size=3200) as ctx:
        ctx.load_histories(h)
        fbp = ctx.initial_fbp(w.n_angles, median_radius=2)
        hull = ctx.hull_detect(wepl_in_mm=1.0, wepl_out_mm=1.0, min_in=1, max_out=0,
                               mask_image=True)
        x = ctx.get_image()
        st = ctx.stats()
    assert st["k"] == 0 and st["steps"] == 0
    np.testing.assert_array_equal(x, np.where(hull == 1, fbp, np.float32(0.0)))
    assert 0 < hull.sum() < hull.size


def test_hull_rejects_bad_parameters():
    w = synth.workload("slice64", n_hist=1000)
    with tvs.Context(w.grid, block_size=64) as ctx:
        with pytest.raises(tvs.TvsError) as e:
            ctx.hull_detect()
        assert e.value.status == tvs.TVS_ESTATE
        ctx.load_histories(w.histories())
        for kw in (dict(min_in=-1), dict(max_out=-2), dict(wepl_in_mm=float("nan"))):
            with pytest.raises(tvs.TvsError) as e:
                ctx.hull_detect(**kw)
            assert e.value.status == tvs.TVS_EINVAL
