"""Pins for the oracle's Bessel/Chebyshev coefficients (Sec. "Chebyshev Polynomials").

Each check uses a route other than the oracle's own formula: the power series
of I_k, Chebyshev-Gauss quadrature of exp(-t(y+1)), the exact values at
y = -1 (lambda = 0, where the heat kernel is the identity) and y = +1, and
finite differences in t.
"""
import math

import numpy as np
import pytest

from oracle import heat


def bessel_i_series(k, t, terms=200):
    """I_k(t) = sum_m (t/2)^(2m+k) / (m! (m+k)!), summed in log space per term."""
    s = 0.0
    for m in range(terms):
        lt = (2 * m + k) * math.log(t / 2.0) - math.lgamma(m + 1) - math.lgamma(m + k + 1)
        s += math.exp(lt)
    return s


def cheb_eval(coef, y):
    """sum' coef_k cos(k arccos y) (b_0 halved), evaluated without the recurrence."""
    th = np.arccos(np.clip(y, -1, 1))
    k = np.arange(len(coef))
    terms = coef[None, :] * np.cos(np.outer(th, k))
    terms[:, 0] *= 0.5
    return terms.sum(axis=1)


@pytest.mark.parametrize("t", [0.5, 1.0, 2.0, 8.0])
def test_coeffs_match_power_series(t):
    K = 30
    b = heat.cheb_coeffs(t, K)
    ref = np.array([2.0 * (-1) ** k * math.exp(-t) * bessel_i_series(k, t) for k in range(K + 1)])
    np.testing.assert_allclose(b, ref, rtol=1e-12, atol=0)


@pytest.mark.parametrize("t", [0.5, 2.0, 8.0])
def test_coeffs_match_chebyshev_gauss_quadrature(t):
    K, N = 40, 4096
    th = np.pi * (np.arange(N) + 0.5) / N
    f = np.exp(-t * (np.cos(th) + 1.0))
    quad = np.array([2.0 / N * np.sum(f * np.cos(k * th)) for k in range(K + 1)])
    np.testing.assert_allclose(heat.cheb_coeffs(t, K), quad, rtol=1e-10, atol=1e-15)


@pytest.mark.parametrize("t,K", [(1.0, 20), (0.5, 30), (2.0, 30), (8.0, 30), (2.0, 40), (2.0, 50)])
def test_truncation_error_within_tail(t, K):
    b = heat.cheb_coeffs(t, K)
    tail = heat.tail_bound(t, K)
    y = np.linspace(-1, 1, 2001)
    err = np.abs(cheb_eval(b, y) - np.exp(-t * (y + 1.0)))
    assert err.max() <= tail + 1e-14
    # lambda = 0 (y = -1) is where H_t x = x for x constant
    p0 = 0.5 * b[0] + np.sum(b[1:] * (-1.0) ** np.arange(1, K + 1))
    assert abs(p0 - 1.0) <= tail + 1e-15
    p1 = 0.5 * b[0] + np.sum(b[1:])
    assert abs(p1 - math.exp(-2 * t)) <= tail + 1e-15


def test_tail_is_small_at_workload_orders():
    # the truncation error at every configuration the library is run at
    for t, K in [(1.0, 20), (0.5, 30), (2.0, 30), (8.0, 30), (2.0, 40), (2.0, 50)]:
        assert heat.tail_bound(t, K) < 1e-17
    # and the bound is not vacuous: low orders have a visible tail
    assert heat.tail_bound(8.0, 5) > 1e-3


@pytest.mark.parametrize("t", [0.5, 2.0, 8.0])
def test_coeff_derivative_matches_finite_difference(t):
    K, h = 40, 1e-6
    fd = (heat.cheb_coeffs(t + h, K) - heat.cheb_coeffs(t - h, K)) / (2 * h)
    np.testing.assert_allclose(heat.cheb_coeffs_dt(t, K), fd, rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("t", [0.5, 2.0])
def test_coeff_derivative_series_is_dt_of_exponential(t):
    K = 50
    y = np.linspace(-1, 1, 501)
    got = cheb_eval(heat.cheb_coeffs_dt(t, K), y)
    np.testing.assert_allclose(got, -(y + 1.0) * np.exp(-t * (y + 1.0)), atol=1e-13)


def test_first_coefficients_at_t1_from_series():
    # b_0..b_5 at t = 1 from the power series, written out to 8 digits
    ref = [0.93151922, -0.41582083, 0.09987755, -0.01631062, 0.00201386, -0.00019973]
    np.testing.assert_allclose(heat.cheb_coeffs(1.0, 5), ref, atol=6e-9)
