"""GPU parity of the initial iterate (tvs_initial_fbp): filtered
backprojection of the binned histories and the in-slice median, against the
oracle's implementation of the same reading (the paper's initial iterate
with a radius-2 median, Section V-A).

Both sides evaluate the same float64 operations in the same order (bin sums
as integers, fixed summation orders, the same cos/sin of the beam angles),
so the float32 images must agree to within one float32 rounding (1e-6
relative, floor 0.1); in practice they are identical.  Cases: the 2-D slice
phantom with the paper's radius 2, a 3-D grid with radius 1 and no
clipping, an odd-sized grid with a non-default bin width, and the radius-0
(no median) form.
"""
import numpy as np
import pytest

import oracle
from paper_1803_01112_amd import synth, tvs

pytestmark = pytest.mark.gpu


def rel_err(x, ref):
    return float(np.max(np.abs(np.asarray(x, np.float64) - ref) / np.maximum(np.abs(ref), 0.1)))


def fbp_both(w, h, A, tau, median_r, clip, grid=None):
    g = grid or w.grid
    print(f"fbp: {w.name} {len(h['ex'])} histories, A={A}, tau={tau}, r={median_r}, clip={clip}",
          flush=True)
    with tvs.Context(g, block_size=256, path_mode="otf") as ctx:
        ctx.load_histories(h)
        img = ctx.initial_fbp(A, median_radius=median_r, t_bin_mm=tau or 0.0, clip_negative=clip)
        back = ctx.get_image()
    want = oracle.fbp_initial(g, h, A, tau=tau, median_r=median_r, clip=clip)
    return img, back, want


def test_slice_phantom_radius_2():
    w = synth.workload("slice64")
    h = w.histories()
    img, back, want = fbp_both(w, h, w.n_angles, None, 2, True)
    assert rel_err(img, want) <= 1e-6
    assert np.array_equal(img, back)                    # it became the context image
    assert np.mean(img == want.astype(np.float32)) > 0.999


def test_volume_radius_1_unclipped():
    w = synth.workload("vol64", n_hist=200_000)
    h = w.histories()
    img, _, want = fbp_both(w, h, w.n_angles, None, 1, False)
    assert (want < 0).any()                              # ringing kept without the clip
    assert rel_err(img, want) <= 1e-6


def test_odd_grid_and_bin_width_no_median():
    w = synth.workload("vol64", n_hist=100_000)
    h = w.histories()
    g = synth.Grid(61, 37, 3, 0.8, 1.1, 2.5, -24.4, -20.35, -3.75)
    img, _, want = fbp_both(w, h, w.n_angles, 0.7, 0, True, grid=g)
    assert rel_err(img, want) <= 1e-6


def test_rejects_bad_parameters():
    w = synth.workload("slice64", n_hist=1000)
    with tvs.Context(w.grid, block_size=64) as ctx:
        with pytest.raises(tvs.TvsError):
            ctx.initial_fbp(90)                          # before load_histories
        ctx.load_histories(w.histories())
        for kw in (dict(n_angles=0), dict(n_angles=90, median_radius=3),
                   dict(n_angles=90, t_bin_mm=-1.0)):
            with pytest.raises(tvs.TvsError):
                ctx.initial_fbp(**kw)
