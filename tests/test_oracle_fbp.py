"""Pins of the oracle's initial iterate: binning of histories, the Ram-Lak
filter, backprojection and the in-slice median (the paper starts from a
median-filtered initial iterate, radius 2, Section V-A; the backprojection
follows the textbook parallel-beam form, see the oracle's header).

Pinned by: the filter's impulse response against the kernel's closed form,
the reconstruction of a uniform disk from its analytic projections (centred
and off-centre, so scale, orientation and interpolation are all fixed),
histories built on known lines landing in their bins with exact mean WEPL,
the median against a brute-force window median, and the full chain on the
synthetic slice phantom approaching its true RSP map.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1803_01112_amd import synth
from paper_1803_01112_amd.synth import Grid


def test_filter_impulse_response():
    nt, tau = 33, 0.7
    for s in (0, 10, 16, 32):
        p = np.zeros(nt)
        p[s] = 1.0
        q = oracle.fbp_filter(p, nt, tau)
        for m in range(nt):
            n = m - s
            h = 1 / (4 * tau * tau) if n == 0 else (
                -1 / (n * n * math.pi ** 2 * tau * tau) if n % 2 else 0.0)
            assert q[m] == pytest.approx(tau * h, rel=1e-14, abs=1e-300)


def disk_projections(A, nz, nt, tau, R, mu, cx=0.0, cy=0.0):
    """p(a, k, m) of a uniform disk (radius R, value mu, centre (cx, cy))."""
    p = np.zeros((A, nz, nt))
    for a in range(A):
        phi = 2 * math.pi * a / A
        tc = -cx * math.sin(phi) + cy * math.cos(phi)      # the centre's lateral coordinate
        t = (np.arange(nt) - nt / 2 + 0.5) * tau - tc
        p[a, :, :] = np.where(np.abs(t) < R, 2 * mu * np.sqrt(np.maximum(R * R - t * t, 0)), 0.0)
    return p.ravel()


@pytest.mark.parametrize("cx,cy", [(0.0, 0.0), (6.0, -4.0)])
def test_disk_reconstruction(cx, cy):
    g = synth.centered_grid(96, 96, 2, 0.5, 0.5, 1.0)
    A, tau, R, mu = 360, 0.5, 15.0, 1.3
    nt = oracle.fbp_lateral_bins(g, tau)
    q = oracle.fbp_filter(disk_projections(A, g.nz, nt, tau, R, mu, cx, cy), nt, tau)
    x = oracle.fbp_backproject(g, q, A, tau, nt).reshape(g.nz, g.ny, g.nx)
    X = g.ox + (np.arange(g.nx) + 0.5) * g.vx
    Y = g.oy + (np.arange(g.ny) + 0.5) * g.vy
    XX, YY = np.meshgrid(X, Y)
    rr = np.hypot(XX - cx, YY - cy)
    for k in range(g.nz):
        inner = x[k][rr < R - 2.0]
        outer = x[k][rr > R + 4.0]
        assert abs(inner.mean() - mu) < 0.01 * mu
        assert np.abs(inner - mu).max() < 0.05 * mu
        # ringing of the sampled edge stays small away from it
        assert np.abs(outer).mean() < 0.02 * mu
        assert np.abs(outer).max() < 0.1 * mu
        # the disk's mass and centre (a half-bin or sign slip moves them)
        near = rr < R + 4.0
        xk = np.where(near, x[k], 0.0)
        assert xk.sum() * g.vx * g.vy == pytest.approx(math.pi * R * R * mu, rel=0.02)
        assert (xk * XX).sum() / xk.sum() == pytest.approx(cx, abs=0.1)
        assert (xk * YY).sum() / xk.sum() == pytest.approx(cy, abs=0.1)


def line_history(phi, t, v, wepl, u_in=-60.0, u_out=55.0, slope=0.0):
    """A history on the straight line at lateral t, height v, beam angle phi."""
    ux, uy = math.cos(phi), math.sin(phi)
    tx, ty = -uy, ux
    e = (u_in * ux + t * tx, u_in * uy + t * ty, v)
    q = (u_out * ux + t * tx, u_out * uy + t * ty, v)
    return dict(ex=e[0], ey=e[1], ez=e[2], qx=q[0], qy=q[1], qz=q[2], eth=slope, eps=0.0,
                qth=slope, qps=0.0, ux=ux, uy=uy, wepl=wepl)


def as_hist(rows):
    return {k: np.array([r[k] for r in rows], np.float32) for k in oracle.HIST_FIELDS}


def test_binning_lands_in_known_bins():
    g = Grid(40, 40, 4, 1.0, 1.0, 2.5, -20.0, -20.0, -5.0)
    A, tau = 8, 1.0
    nt = oracle.fbp_lateral_bins(g, tau)
    rows = [line_history(2 * math.pi * 3 / A, 4.25, 1.0, 10.0),      # a 3, slice 2, m nt/2+4
            line_history(2 * math.pi * 3 / A, 4.75, 1.0, 14.0),      # same bin
            line_history(2 * math.pi * 7 / A, -0.5, -4.0, 7.0),      # a 7, slice 0, m nt/2-1
            line_history(2 * math.pi * 7 / A, 0.0, 9.0, 5.0),        # above the grid: dropped
            line_history(0.0, 0.3, 0.2, 9.0, u_in=10.0, u_out=10.0)]  # no length: dropped
    p, cnt = oracle.fbp_bin(g, as_hist(rows), A, tau, nt)
    p = p.reshape(A, g.nz, nt)
    cnt = cnt.reshape(A, g.nz, nt)
    assert cnt.sum() == 3
    assert cnt[3, 2, nt // 2 + 4] == 2 and p[3, 2, nt // 2 + 4] == 12.0
    assert cnt[7, 0, nt // 2 - 1] == 1 and p[7, 0, nt // 2 - 1] == 7.0
    # the crossing of u = 0, not the entry point, decides: a tilted line
    phi = 2 * math.pi * 1 / A
    h = line_history(phi, 2.5, 0.0, 3.0)
    h["ez"], h["qz"] = -3.0, 3.0                      # height 0 at u = 0 (entry -60, exit +55)
    p2, cnt2 = oracle.fbp_bin(g, as_hist([h]), A, tau, nt)
    k0 = int(math.floor((-3.0 + 6.0 * 60.0 / 115.0 + 5.0) / 2.5))
    assert cnt2.reshape(A, g.nz, nt)[1, k0, nt // 2 + 2] == 1


def test_median_brute_force():
    rng = np.random.default_rng(5)
    g = Grid(9, 7, 2, 1.0, 1.0, 1.0, 0, 0, 0)
    x = rng.normal(size=g.nvox)
    for r in (1, 2):
        y = oracle.median_slices(g, x, r).reshape(g.nz, g.ny, g.nx)
        v = x.reshape(g.nz, g.ny, g.nx)
        for k in range(g.nz):
            for j in range(g.ny):
                for i in range(g.nx):
                    win = np.sort(v[k, max(0, j - r):j + r + 1, max(0, i - r):i + r + 1].ravel())
                    assert y[k, j, i] == win[(win.size - 1) // 2]


def test_full_chain_on_the_slice_phantom():
    w = synth.workload("slice64")
    h = w.histories()
    x = oracle.fbp_initial(w.grid, h, w.n_angles, median_r=2)
    truth = synth.truth_image(w.grid, w.phantom).astype(np.float64)
    X = w.grid.ox + (np.arange(w.grid.nx) + 0.5) * w.grid.vx
    XX, YY = np.meshgrid(X, X)
    rr = np.hypot(XX, YY).ravel()
    inside = rr < 0.5 * w.diameter - 6.0
    outside = rr > 0.5 * w.diameter + 6.0
    # background and inserts recovered to a few percent of RSP 1, zero outside
    assert np.mean(np.abs(x[inside] - truth[inside])) < 0.05
    assert np.max(np.abs(x[outside])) < 0.1
