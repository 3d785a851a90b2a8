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
    keep = w > lanczos.REL_WEIGHT * w.sum()
    mu_min, mu_max = lanczos.support_estimate(a, b, n0)
    assert abs(mu_min - lam[keep].min()) < 1e-10
    assert abs(mu_max - lam[keep].max()) < 1e-10
    # what falls below the cut-off is rounding: the zero-weight eigenspaces
    assert np.all(w[~keep] < 1e-26 * w.sum())


def test_small_weight_extreme_node_is_support():
    """A random 7 x 9 map (no symmetry: simple eigenvalues).  The applied
    field e0 = (cos t, sin t) is turned until the top eigenvalue of the dense
    Gamma_1 chi Gamma_1 carries a weight of about 1e-10 of the total: that
    eigenvalue still belongs to the support, and the estimate must return it
    (a cut-off of 1e-6 would drop it)."""
    chi = inputs.random_phase((7, 9), 0.4, seed=4)
    d, m = 2, chi.size
    G = dense.gamma_dense(chi.shape, "rotated")
    X = np.diag(np.tile(chi.ravel().astype(float), d))
    lam, phi = np.linalg.eigh(G @ X @ G)
    ux = phi.conj().T @ (G @ (X @ np.concatenate([np.ones(m), np.zeros(m)])))
    uy = phi.conj().T @ (G @ (X @ np.concatenate([np.zeros(m), np.ones(m)])))
    tot = np.abs(ux) ** 2 + np.abs(uy) ** 2
    top = int(np.flatnonzero(tot > 1e-12 * tot.sum()).max())
    assert lam[top] < 1 - 1e-6 and abs(lam[top] - lam[top - 1]) > 1e-6
    t0 = np.arctan2(-ux[top].real, uy[top].real)      # weight of lam[top] vanishes at t0
    t = t0 + 1e-4
    e0 = (np.cos(t), np.sin(t))
    w = np.abs(np.cos(t) * ux + np.sin(t) * uy) ** 2
    rel = w[top] / w.sum()
    assert 1e-12 < rel < 1e-8
    a, b, n0 = lanczos.lanczos(chi, e0, d * m, "rotated")
    mu_min, mu_max = lanczos.support_estimate(a, b, n0)
    assert abs(mu_max - lam[top]) < 1e-9
    # the old 1e-6 cut-off would have returned the next node instead
    assert lanczos.support_estimate(a, b, n0, rel_weight=1e-6)[1] < lam[top] - 1e-6


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
