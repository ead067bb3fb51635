"""Pins of the oracle's most-likely-path (MLP) model.

The paper (arXiv 1803.01112, Section I) names the MLP of each proton but
prints no MLP value.  The oracle uses the Fermi-Eyges / Highland form: a
Gaussian multiple-scattering model whose angular variance grows with depth
as E0^2 (1 + 0.038 ln(d/X0))^2 / X0 * integral of 1/(beta^2 p^2), conditioned
on the measured entry and exit states.  These tests pin it against what
does not depend on the oracle's own code:
  * numerical quadrature of the defining moment integrals;
  * the covariance form of Gaussian conditioning (numpy), fed with those
    quadrature moments, for the vertex position;
  * the straight chord for collinear entry/exit states;
  * the cubic Hermite interpolant for constant scattering power and no
    log term (posterior mean of integrated Brownian motion);
  * symmetry under reversal of the path (constant power);
  * relativistic kinematics of the tabulated 1/(beta^2 p^2).
Absolute physical realism of the coefficient table beyond these checks is
parity unpinned (no printed MLP values exist).
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle

E0, X0 = 13.6, 360.8          # MeV, mm
MP = 938.272                  # proton mass, MeV


def scattering_power(w_mm, const_power=False):
    """1/(beta^2 p^2) in MeV^-2 at depth w (mm), from the published per-cm table."""
    a = [7.457e-6, 4.548e-7, -5.777e-8, 1.301e-8, -9.228e-10, 2.687e-11]
    if const_power:
        return a[0]
    w = w_mm / 10.0
    return sum(c * w ** k for k, c in enumerate(a))


def quad_sigmas(d1, L, log_term=True, const_power=False):
    P = lambda w: scattering_power(w, const_power)

    def A(d):
        f = 1.0 + 0.038 * math.log(d / X0) if log_term else 1.0
        return E0 * E0 * f * f / X0

    q = lambda fn, a, b: integrate.quad(fn, a, b, epsabs=0, epsrel=1e-13, limit=200)[0]
    s1 = [q(lambda w: (d1 - w) ** m * P(w), 0.0, d1) for m in (2, 1, 0)]
    s2 = [q(lambda w: (L - w) ** m * P(w), d1, L) for m in (2, 1, 0)]
    A1, A2 = A(d1), A(L - d1)
    S1 = A1 * np.array([[s1[0], s1[1]], [s1[1], s1[2]]])
    S2 = A2 * np.array([[s2[0], s2[1]], [s2[1], s2[2]]])
    return S1, S2


@pytest.mark.parametrize("d1,L", [(1.0, 150.0), (37.5, 150.0), (75.0, 150.0), (149.0, 150.0),
                                  (10.0, 40.0), (96.0, 192.0)])
@pytest.mark.parametrize("log_term", [True, False])
def test_moments_match_quadrature(d1, L, log_term):
    S1, S2 = oracle.mlp_sigmas(d1, L, log_term=log_term)
    Q1, Q2 = quad_sigmas(d1, L, log_term=log_term)
    np.testing.assert_allclose(S1, Q1, rtol=1e-9, atol=0)
    np.testing.assert_allclose(S2, Q2, rtol=1e-9, atol=0)


def test_scattering_power_kinematics():
    """P(0) is 1/(beta^2 p^2) of a 200 MeV proton; deeper values follow the
    residual energy of a Bragg-Kleeman range-energy rule within 6 %."""
    def inv_b2p2(T):
        pc2 = T * T + 2 * T * MP
        E = T + MP
        return 1.0 / (pc2 * pc2 / (E * E))

    assert scattering_power(0.0) == pytest.approx(inv_b2p2(200.0), rel=0.01)
    r0 = 0.0022 * 200.0 ** 1.77 * 10.0     # mm
    for w in (50.0, 100.0, 150.0, 200.0):
        T = ((r0 - w) / 10.0 / 0.0022) ** (1 / 1.77)
        assert scattering_power(w) == pytest.approx(inv_b2p2(T), rel=0.06)
    ws = np.linspace(0, 200, 41)
    assert np.all(np.diff([scattering_power(w) for w in ws]) > 0)


@pytest.mark.parametrize("L", [20.0, 150.0, 250.0])
def test_sigmas_positive_definite(L):
    for d1 in np.linspace(1.0, L - 1.0, 23):
        S1, S2 = oracle.mlp_sigmas(d1, L)
        for S in (S1, S2):
            assert S[0, 0] > 0 and S[1, 1] > 0
            assert np.linalg.det(S) > 0


def _hist(entry, exit_, th0, ps0, th2, ps2, u):
    return [entry[0], entry[1], entry[2], exit_[0], exit_[1], exit_[2], th0, ps0, th2, ps2,
            u[0], u[1]]


def _frame(u):
    u = np.asarray(u, float) / np.hypot(*u)
    t = np.array([-u[1], u[0]])
    return u, t


def test_vertex_matches_covariance_form_conditioning():
    """Vertex = E[state at d1 | entry, exit] computed in covariance form from
    quadrature moments (an algebraically different route to the same value)."""
    rng = np.random.default_rng(7)
    for _ in range(6):
        phi = rng.uniform(0, 2 * np.pi)
        u, tdir = _frame((math.cos(phi), math.sin(phi)))
        L = rng.uniform(60, 180)
        t0, t2 = rng.uniform(-30, 30), rng.uniform(-30, 30)
        v0, v2 = rng.uniform(-5, 5), rng.uniform(-5, 5)
        th0, th2, ps0, ps2 = rng.normal(0, 0.03, 4)
        u0 = rng.uniform(-90, -30)
        p_in = np.r_[u0 * u + t0 * tdir, v0]
        p_out = np.r_[(u0 + L) * u + t2 * tdir, v2]
        step = 7.0
        pts = oracle.mlp_polyline(_hist(p_in, p_out, th0, ps0, th2, ps2, u), step)
        J = int(math.ceil(L / step))
        assert len(pts) == J + 1
        np.testing.assert_array_equal(pts[0], p_in)
        np.testing.assert_array_equal(pts[-1], p_out)
        for j in (1, J // 2, J - 1):
            d1 = j * step
            d2 = L - d1
            S1, S2 = quad_sigmas(d1, L)
            R0 = np.array([[1, d1], [0, 1.0]])
            R1 = np.array([[1, d2], [0, 1.0]])
            C12 = S1 @ R1.T
            C22 = R1 @ S1 @ R1.T + S2
            y = []
            for y0, y2 in (((t0, th0), (t2, th2)), ((v0, ps0), (v2, ps2))):
                m1 = R0 @ np.array(y0)
                m2 = R1 @ m1
                y.append(m1 + C12 @ np.linalg.solve(C22, np.array(y2) - m2))
            ud = u0 + d1
            want = np.r_[ud * u + y[0][0] * tdir, y[1][0]]
            np.testing.assert_allclose(pts[j], want, rtol=0, atol=1e-7)


def test_collinear_states_give_straight_chord():
    rng = np.random.default_rng(3)
    for _ in range(10):
        phi = rng.uniform(0, 2 * np.pi)
        u, tdir = _frame((math.cos(phi), math.sin(phi)))
        L = rng.uniform(20, 200)
        t0, t2 = rng.uniform(-40, 40, 2)
        v0, v2 = rng.uniform(-10, 10, 2)
        th = (t2 - t0) / L
        ps = (v2 - v0) / L
        u0 = -L / 2
        p_in = np.r_[u0 * u + t0 * tdir, v0]
        p_out = np.r_[(u0 + L) * u + t2 * tdir, v2]
        for lt in (True, False):
            pts = oracle.mlp_polyline(_hist(p_in, p_out, th, ps, th, ps, u), 1.0, log_term=lt)
            d = p_out - p_in
            for p in pts[1:-1]:
                s = np.dot(p - p_in, d) / np.dot(d, d)
                np.testing.assert_allclose(p, p_in + s * d, rtol=0, atol=1e-12 * L)


def test_constant_power_gives_cubic_hermite():
    rng = np.random.default_rng(11)
    for _ in range(8):
        L = float(rng.integers(40, 200))
        t0, t2, v0, v2 = rng.uniform(-20, 20, 4)
        th0, th2, ps0, ps2 = rng.normal(0, 0.05, 4)
        p_in = np.array([-L / 2, t0, v0])
        p_out = np.array([L / 2, t2, v2])
        pts = oracle.mlp_polyline(_hist(p_in, p_out, th0, ps0, th2, ps2, (1.0, 0.0)), 1.0,
                                  log_term=False, const_power=True)
        for j in range(1, len(pts) - 1):
            s = j / L
            h00, h10 = 2 * s ** 3 - 3 * s ** 2 + 1, s ** 3 - 2 * s ** 2 + s
            h01, h11 = -2 * s ** 3 + 3 * s ** 2, s ** 3 - s ** 2
            t = h00 * t0 + h10 * L * th0 + h01 * t2 + h11 * L * th2
            v = h00 * v0 + h10 * L * ps0 + h01 * v2 + h11 * L * ps2
            np.testing.assert_allclose(pts[j], [-L / 2 + j, t, v], rtol=0, atol=1e-9)


def test_reversal_symmetry_constant_power():
    rng = np.random.default_rng(5)
    for _ in range(6):
        L = 120.0
        t0, t2, v0, v2 = rng.uniform(-20, 20, 4)
        th0, th2, ps0, ps2 = rng.normal(0, 0.05, 4)
        a = np.array([-60.0, t0, v0])
        b = np.array([60.0, t2, v2])
        fwd = oracle.mlp_polyline(_hist(a, b, th0, ps0, th2, ps2, (1.0, 0.0)), 1.0,
                                  const_power=True)
        # reversed: beam axis -x, lateral axis -y; dt'/du' = dt/du, dv/du' = -dv/du
        rev = oracle.mlp_polyline(_hist(b, a, th2, -ps2, th0, -ps0, (-1.0, 0.0)), 1.0,
                                  const_power=True)
        np.testing.assert_allclose(rev[::-1], fwd, rtol=0, atol=1e-9)


def test_no_row_when_exit_not_deeper():
    h = [10.0, 0, 0, -10.0, 0, 0, 0, 0, 0, 0, 1.0, 0.0]
    assert oracle.mlp_polyline(h, 1.0) is None
    h = [10.0, 0, 0, 10.0, 5.0, 0, 0, 0, 0, 0, 1.0, 0.0]
    assert oracle.mlp_polyline(h, 1.0) is None


def test_short_path_has_no_interior_vertex():
    h = [0.0, 0, 0, 0.5, 0.1, 0, 0, 0, 0, 0, 1.0, 0.0]
    pts = oracle.mlp_polyline(h, 1.0)
    assert len(pts) == 2


def test_oracle_log_against_the_math_library():
    """The Highland factor's logarithm (written out in the oracle from the
    atanh series) agrees with the C library's to a few ulp over the depths
    the MLP evaluates (d / X0 from 1e-7 to 3), across the reduction's
    boundary at sqrt(1/2) and at exact powers of two."""
    rng = np.random.default_rng(2)
    xs = np.concatenate([np.exp(rng.uniform(np.log(1e-7), np.log(3.0), 20000)),
                         [0.5, 1.0, 2.0, 0.25, 2.0 ** -20],
                         np.nextafter(math.sqrt(0.5), 0.0) * np.array([1.0, 1.0 + 1e-15]),
                         [math.sqrt(0.5), 1.0 - 1e-15, 1.0 + 1e-15]])
    worst = 0.0
    for x in xs:
        got, want = oracle.log(float(x)), math.log(float(x))
        ulp = max(np.spacing(abs(want)), np.spacing(1e-300))
        if want != 0.0:
            worst = max(worst, abs(got - want) / ulp)
        else:
            assert got == 0.0
    assert worst <= 4.0, worst
