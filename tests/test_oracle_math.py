"""Pins of the oracle's changeover functions K and W (Section 2.1).

K is pinned by the paper's own characterisation: the lowest-order polynomial
in x with K(0)=0, K(1)=1 and derivatives up to third order vanishing at both
ends -- eight conditions that fix a degree-7 polynomial uniquely.  W is pinned
by the defining relation K = W - s dW/ds with W = 1 beyond the outer cutoff,
integrated by adaptive quadrature (independent of the closed form the oracle
evaluates).
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

GAMMAS = [0.1, 0.05, 0.3]


def _x_to_y(x, g):
    return g + x * (1.0 - g)


@pytest.mark.parametrize("g", GAMMAS)
def test_K_is_the_unique_C3_polynomial(oracle_lib, g):
    xs = np.linspace(0.0, 1.0, 41)[:-1]
    ks = oracle_lib.K(_x_to_y(xs, g), g)
    coef = np.polyfit(xs, ks, 7)
    fit = np.poly1d(coef)
    assert np.max(np.abs(fit(xs) - ks)) < 1e-12          # a degree-7 polynomial in x
    assert abs(fit(0.0)) < 1e-12 and abs(fit(1.0) - 1.0) < 1e-10
    for order in (1, 2, 3):
        d = fit.deriv(order)
        assert abs(d(0.0)) < 1e-8, order
        assert abs(d(1.0)) < 1e-8, order


@pytest.mark.parametrize("g", GAMMAS)
def test_K_piecewise_ends_and_symmetry(oracle_lib, g):
    assert oracle_lib.K(0.0, g) == 0.0
    assert oracle_lib.K(g * 0.999, g) == 0.0
    assert oracle_lib.K(g, g) == 0.0
    assert oracle_lib.K(1.0, g) == 1.0
    assert oracle_lib.K(5.0, g) == 1.0
    assert abs(oracle_lib.K(_x_to_y(0.5, g), g) - 0.5) < 1e-15
    xs = np.linspace(0.01, 0.99, 57)
    k1 = oracle_lib.K(_x_to_y(xs, g), g)
    k2 = oracle_lib.K(_x_to_y(1.0 - xs, g), g)
    np.testing.assert_allclose(k1 + k2, 1.0, atol=1e-14)
    assert np.all(np.diff(k1) > 0)


@pytest.mark.parametrize("g", GAMMAS)
def test_dK_matches_finite_difference(oracle_lib, g):
    ys = _x_to_y(np.linspace(0.02, 0.98, 25), g)
    hstep = 1e-6
    fd = (oracle_lib.K(ys + hstep, g) - oracle_lib.K(ys - hstep, g)) / (2 * hstep)
    np.testing.assert_allclose(oracle_lib.dK(ys, g), fd, rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("g", GAMMAS)
def test_W_from_defining_relation(oracle_lib, g):
    """W(y)/y = 1 + int_y^1 K(t)/t^2 dt  (from K = W - y W', W(1) = 1)."""
    ys = np.concatenate([np.linspace(0.0, g, 5, endpoint=False),
                         np.linspace(g, 1.0, 33)[:-1], [1.0, 1.5, 10.0]])
    for y in ys:
        if y >= 1.0:
            ref = 1.0 / y
        else:
            lo = max(y, g)
            integ, _ = quad(lambda t: oracle_lib.K(t, g) / (t * t), lo, 1.0,
                            epsabs=1e-14, epsrel=1e-13, limit=200)
            ref = 1.0 + integ
        got = float(oracle_lib.W_over_y(y, g))
        assert abs(got - ref) <= 1e-12 * abs(ref), (y, got, ref)


@pytest.mark.parametrize("g", GAMMAS)
def test_K_equals_W_minus_yWprime(oracle_lib, g):
    ys = _x_to_y(np.linspace(0.03, 0.97, 23), g)
    hstep = 1e-5
    wp = (oracle_lib.W(ys + hstep, g) - oracle_lib.W(ys - hstep, g)) / (2 * hstep)
    np.testing.assert_allclose(oracle_lib.W(ys, g) - ys * wp, oracle_lib.K(ys, g), atol=1e-9)


@pytest.mark.parametrize("g", GAMMAS)
def test_W_continuous_and_C_slope(oracle_lib, g):
    C = oracle_lib.C_gamma(g)
    d = 1e-12
    assert abs(oracle_lib.W(g - d, g) - oracle_lib.W(g + d, g)) < 1e-10
    assert abs(oracle_lib.W(g, g) - C * g) < 1e-13
    assert abs(oracle_lib.W(1.0 - d, g) - 1.0) < 1e-10
    # slope inside r_in equals the slope W'(gamma+)
    wp = (oracle_lib.W(g + 2e-6, g) - oracle_lib.W(g + 1e-6, g)) / 1e-6
    assert abs(wp - C) < 1e-5


def test_C_limits(oracle_lib):
    # gamma -> 0: C -> 7/3 (the log term vanishes, numerator -> -7, (g-1)^7 -> -1)
    assert abs(oracle_lib.C_gamma(1e-7) - 7.0 / 3.0) < 1e-4
    # C(gamma) = 1 + int_gamma^1 K(t)/t^2 dt
    for g in GAMMAS:
        integ, _ = quad(lambda t: oracle_lib.K(t, g) / (t * t), g, 1.0, epsabs=1e-14, epsrel=1e-13)
        assert abs(oracle_lib.C_gamma(g) - (1.0 + integ)) < 1e-12


def test_direct_module_W_matches_oracle(oracle_lib):
    """The quadrature-based W of the O(N^2) reference agrees with the oracle's closed form."""
    from oracle import direct
    g = 0.1
    ys = np.linspace(0.0, 1.2, 97)
    np.testing.assert_allclose(direct.W_over_y_np(ys, g),
                               oracle_lib.W_over_y(ys, g), rtol=1e-13)
    np.testing.assert_allclose(direct.K_np(ys, g), oracle_lib.K(ys, g), atol=1e-15)
    assert math.isclose(direct.C_np(g), oracle_lib.C_gamma(g), rel_tol=1e-13)
