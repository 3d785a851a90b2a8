"""Pins of the series-coefficient oracle (eqs. J5-J7) and its Pade approximants.

Expected coefficients come from closed forms expanded with plain power-series
arithmetic (laminates: arithmetic and harmonic means; square array: eq. J47a
through a Cauchy integral), not from the oracle's recursion.
"""
import numpy as np
import pytest

from oracle import scalars, series, solver
from paper_2001_08289_amd import inputs


def _ser_mul(a, b, n):
    return np.convolve(a[:n + 1], b[:n + 1])[:n + 1]


def _ser_div(a, b, n):
    """Taylor coefficients of a/b up to z^n (b_0 != 0)."""
    a = np.concatenate([a, np.zeros(n + 1)])[:n + 1].astype(complex)
    b = np.concatenate([b, np.zeros(n + 1)])[:n + 1].astype(complex)
    c = np.zeros(n + 1, complex)
    for k in range(n + 1):
        c[k] = (a[k] - np.dot(b[1:k + 1], c[k - 1::-1][:k])) / b[0]
    return c


def _closed_form_coeffs(mean, alpha, beta, n):
    """c_k of sigma*/sqrt(t) for sigma* = mean(sigma1), by series arithmetic in z.

    sqrt t = (1 + z)/(1 - z); sigma1(t) inverts eq. J6:
    sigma1 = -[(beta - alpha) + beta (1 + alpha)(t - 1)] / [(1 + alpha)(t - 1) - (beta - alpha)].
    """
    one = np.zeros(n + 1)
    one[0] = 1.0
    geo = np.ones(n + 1)                                # 1/(1 - z)
    w = _ser_mul(np.array([1.0, 1.0]), geo, n)          # (1 + z)/(1 - z)
    t = _ser_mul(w, w, n)
    tm1 = t - one
    num = -((beta - alpha) * one + beta * (1 + alpha) * tm1)
    den = (1 + alpha) * tm1 - (beta - alpha) * one
    s1 = _ser_div(num, den, n)
    sig = mean(s1, one, n)
    winv = _ser_div(np.array([1.0, -1.0]), np.array([1.0, 1.0]), n)   # (1 - z)/(1 + z)
    return _ser_mul(sig, winv, n)


@pytest.mark.parametrize("symbol", ["rotated", "spectral", "network"])
@pytest.mark.parametrize("alpha,beta", [(0.25, 4.0), (0.2, 3.0)])
def test_laminate_series_closed_form(symbol, alpha, beta):
    """Layers normal to x: e0 along y sees the arithmetic mean, e0 along x the
    harmonic mean; both are exact for the discrete problem."""
    f = 0.25
    chi = inputs.laminate(16, 2, fraction=f, axis=0)
    # rounding excites the zero-weight modes whose singularities (sigma1 = 0
    # and infinity) sit at |z| ~ 1/3 for these intervals, so the error of c_k
    # grows like 3.5^k; 12 terms keep it below 1e-9 relative
    n = 12
    arith = lambda s1, one, n: one + f * (s1 - one)                                # noqa: E731
    harm = lambda s1, one, n: _ser_div(s1, f * one + (1 - f) * s1, n)             # noqa: E731
    for e0, mean in (((0.0, 1.0), arith), ((1.0, 0.0), harm)):
        got = series.series_coefficients(chi, e0, alpha, beta, n, symbol)
        exp = _closed_form_coeffs(mean, alpha, beta, n)
        assert np.abs(got - exp).max() < 1e-9 * max(1.0, np.abs(exp).max())


def test_square_array_series_matches_j47a_cauchy():
    """Square array at 64^2 (rotated symbol): sigma* equals eq. J47a to ~1e-12,
    so its Taylor coefficients in z (Cauchy integral on |z| = 1/2) pin the
    low-order c_k (higher orders see the small difference between the
    discrete and the continuum spectral measure)."""
    alpha, beta, n = 0.25, 4.0, 7
    chi = inputs.square_array(64)
    got = series.series_coefficients(chi, (1.0, 0.0), alpha, beta, n)
    K, r = 256, 0.5
    zs = r * np.exp(2j * np.pi * np.arange(K) / K)
    s1 = scalars.sigma1_from_z(zs, alpha, beta)
    w = (1 + zs) / (1 - zs)
    f = scalars.obnosov_square_array(s1) / w
    exp = np.array([np.mean(f * zs ** (-k)) for k in range(n + 1)])
    assert np.abs(got - exp).max() < 1e-12


def test_series_sum_matches_accelerated_solve():
    """The partial sum at sigma1 reproduces the accelerated solver's sigma*
    (|z| < 1/3 at these sigma1, where the coefficient noise stays harmless)."""
    alpha, beta = 0.25, 4.0
    chi = inputs.square_array(32)
    c = series.series_coefficients(chi, (1.0, 0.0), alpha, beta, 60)
    for s1 in (10.0, 3 + 2j, 0.05):
        ref = solver.solve(chi, s1, [1, 0], "acc_em", alpha=alpha, beta=beta, tol=1e-14,
                           max_iter=3000)["sigma_star"]
        assert abs(series.evaluate(c, s1, alpha, beta) - ref) < 1e-11 * abs(ref)


def test_pade_exact_for_laminate_and_faster_than_partial_sums():
    """The arithmetic-mean laminate gives sigma*/sqrt(t) rational in z of
    degree 3 over 3, so the [3/3] approximant from 7 coefficients is exact;
    on the square array Pade beats the partial sum of the same length near
    the slit."""
    alpha, beta = 0.25, 4.0
    lam = inputs.laminate(16, 2, fraction=0.25, axis=0)
    c = series.series_coefficients(lam, (0.0, 1.0), alpha, beta, 6)
    a, q = series.pade(c, 3)
    for s1 in (10.0, -0.1 + 0.05j, 1e3):
        exact = 1 + 0.25 * (s1 - 1)
        assert abs(series.evaluate_pade(a, q, s1, alpha, beta) - exact) < 1e-11 * abs(exact)
    chi = inputs.square_array(64)
    c = series.series_coefficients(chi, (1.0, 0.0), alpha, beta, 20)
    a, q = series.pade(c, 10)
    for s1 in (-0.2 + 0.02j, -5.0 + 0.1j):
        exact = scalars.obnosov_square_array(s1)
        e_sum = abs(series.evaluate(c, s1, alpha, beta) - exact)
        e_pade = abs(series.evaluate_pade(a, q, s1, alpha, beta) - exact)
        assert e_pade < e_sum


def test_pade_of_exponential_textbook():
    """[2/2] approximant of exp(z): (1 + z/2 + z^2/12) / (1 - z/2 + z^2/12)."""
    import math
    c = np.array([1.0 / math.factorial(k) for k in range(5)])
    a, q = series.pade(c, 2)
    assert np.allclose(a, [1.0, 0.5, 1.0 / 12.0], atol=1e-14)
    assert np.allclose(q, [1.0, -0.5, 1.0 / 12.0], atol=1e-14)
