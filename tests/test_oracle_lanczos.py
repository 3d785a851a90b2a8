"""Pins of the Lanczos support estimate (oracle): a dense eigen-decomposition
of Gamma_1 chi Gamma_1 (explicit DFT matrices, numpy.linalg.eigh), the
one-point measure of a laminate, and the power iteration."""
import numpy as np
import pytest

from oracle import dense, interval, lanczos
from paper_2001_08289_amd import inputs


@pytest.mark.parametrize("symbol", ["rotated", "spectral", "network"])
def test_gauss_rule_matches_dense_spectral_measure(symbol):
    chi = inputs.random_phase((6, 8), 0.35, seed=2)
    d, m = 2, chi.size
    G = dense.gamma_dense(chi.shape, symbol)
    X = np.diag(np.tile(chi.ravel().astype(float), d))
    A = G @ X @ G
    e0 = np.concatenate([np.ones(m), np.zeros(m)])
    v0 = G @ (X @ e0)
    lam, phi = np.linalg.eigh(A)
    w = np.abs(phi.conj().T @ v0) ** 2
    a, b, n0 = lanczos.lanczos(chi, (1.0, 0.0), d * m, symbol)
    theta, wts = lanczos.gauss_rule(a, b, n0)
    assert abs(n0 - np.vdot(v0, v0).real) < 1e-10 * n0
    # the Gauss rule of the full Krylov space reproduces every moment
    for k in range(0, 2 * len(a)):
        mk = np.sum(w * lam ** k)
        assert abs(np.sum(wts * theta ** k) - mk) < 1e-9 * max(1.0, abs(mk)) * n0
    keep = w > 1e-6 * w.sum()
    mu_min, mu_max = lanczos.support_estimate(a, b, n0)
    assert abs(mu_min - lam[keep].min()) < 1e-10
    assert abs(mu_max - lam[keep].max()) < 1e-10


def test_laminate_measure_is_one_point():
    """Layers normal to x, e0 = e_x: Gamma_1 chi e_x = (chi - f) e_x and
    Gamma_1 chi (chi - f) e_x = (1 - f)(chi - f) e_x, so the measure is the
    single point 1 - f with weight N^d f (1 - f)."""
    f = 0.25
    chi = inputs.laminate(16, 2, fraction=f, axis=0)
    a, b, n0 = lanczos.lanczos(chi, (1.0, 0.0), 10)
    theta, wts = lanczos.gauss_rule(a, b, n0)
    assert len(a) == 1
    assert abs(theta[0] - (1 - f)) < 1e-13
    assert abs(wts[0] - chi.size * f * (1 - f)) < 1e-10 * chi.size


def test_square_array_support_and_power_iteration():
    """Square array at 25%: the continuum support is [1/4, 3/4]; the extreme
    Gauss nodes agree with the power iteration's extreme eigenvalues."""
    chi = inputs.square_array(64)
    alpha, beta, alpha_u, beta_u, mu_min, mu_max = lanczos.interval(chi, (1.0, 0.0), 60)
    assert 0.245 < mu_min < 0.2505 and 0.74 < mu_max < 0.7505
    pa, pb, pmin, pmax = interval.estimate_interval(chi, 100)
    assert abs(mu_max - pmax) < 2e-3 and abs(mu_min - pmin) < 2e-3
    assert abs(alpha_u * beta_u - 1.0) < 1e-14 and alpha_u <= alpha + 1e-15
