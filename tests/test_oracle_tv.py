"""Pins of the oracle's total variation and its subgradient.

phi = TV, the local variations added over every voxel (arXiv 1803.01112,
Section IV); v = -grad phi/||grad phi|| (Appendix A).  Reading: per slice,
isotropic forward differences, zero difference past the last row/column,
local variation m = sqrt(dx^2 + dy^2 + eps^2), phi = sum (m - eps).
Pinned by: zero on constant images, the closed form of a step edge,
additivity over slices, and central finite differences of phi.
"""
import numpy as np
import pytest

import oracle
from paper_1803_01112_amd.synth import Grid

G3 = Grid(9, 7, 3, 1.0, 1.0, 2.5, 0, 0, 0)


def test_zero_on_constant_image():
    x = np.full(G3.nvox, 1.7)
    assert oracle.tv(G3, x) == 0.0
    g, n2 = oracle.tv_grad(G3, x)
    assert n2 == 0.0 and np.all(g == 0.0)
    assert oracle.tv(G3, x, eps=0.3) == pytest.approx(0.0, abs=1e-15)


@pytest.mark.parametrize("h", [1.0, -0.25, 3.5])
def test_step_edges(h):
    x = np.zeros((G3.nz, G3.ny, G3.nx))
    x[:, :, 4:] = h                                  # jump along x
    assert oracle.tv(G3, x.ravel()) == pytest.approx(abs(h) * G3.ny * G3.nz, rel=1e-15)
    y = np.zeros((G3.nz, G3.ny, G3.nx))
    y[:, 3:, :] = h                                  # jump along y
    assert oracle.tv(G3, y.ravel()) == pytest.approx(abs(h) * G3.nx * G3.nz, rel=1e-15)
    z = np.zeros((G3.nz, G3.ny, G3.nx))
    z[1:, :, :] = h                                  # jump along z: no in-slice variation
    assert oracle.tv(G3, z.ravel()) == 0.0


def test_additive_over_slices():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(G3.nz, G3.ny, G3.nx))
    g1 = Grid(G3.nx, G3.ny, 1, 1.0, 1.0, 2.5, 0, 0, 0)
    total = sum(oracle.tv(g1, x[k].ravel()) for k in range(G3.nz))
    assert oracle.tv(G3, x.ravel()) == pytest.approx(total, rel=1e-14)


def central_differences(grid, x, eps, h=1e-6):
    g = np.zeros_like(x)
    for j in range(x.size):
        xp = x.copy()
        xm = x.copy()
        xp[j] += h
        xm[j] -= h
        g[j] = (oracle.tv(grid, xp, eps) - oracle.tv(grid, xm, eps)) / (2 * h)
    return g


@pytest.mark.parametrize("eps", [0.0, 0.05])
def test_gradient_matches_finite_differences(eps):
    rng = np.random.default_rng(1)
    x = rng.uniform(0.5, 1.5, G3.nvox)
    g, n2 = oracle.tv_grad(G3, x, eps)
    fd = central_differences(G3, x, eps)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-7)
    assert n2 == pytest.approx(float(g @ g), rel=1e-14)


def test_gradient_with_smoothing_on_flat_image():
    x = np.ones(G3.nvox)
    x[10] = 1.2
    g, _ = oracle.tv_grad(G3, x, 0.1)
    fd = central_differences(G3, x, 0.1)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-7)


def test_descent_direction_decreases_tv():
    rng = np.random.default_rng(2)
    x = rng.uniform(0.5, 1.5, G3.nvox)
    g, n2 = oracle.tv_grad(G3, x)
    v = -g / np.sqrt(n2)
    assert oracle.tv(G3, x + 1e-4 * v) < oracle.tv(G3, x)
