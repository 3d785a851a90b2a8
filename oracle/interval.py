"""Power-iteration estimate of the singularity interval [-beta, -alpha] (oracle).

sigma*(sigma1) is singular where sigma1 = 1 - 1/mu for mu in the spectrum of
Gamma_1 chi Gamma_1 on E (the resolvent behind the series of eq. J0-0).  The
paper only needs estimates of alpha and beta (section "Estimating the
parameters alpha and beta"); here they come from the extreme eigenvalues:
  alpha = 1/mu_max - 1,   beta = 1/mu_min - 1,
with mu_max the top of Gamma_1 chi Gamma_1 and 1 - mu_min the top of
Gamma_1 (1 - chi) Gamma_1 (the two add up to the identity on E).

Sequence (identical on both sides): u_0 = e0, u_k = Gamma_1(w u_{k-1}) for
k = 1 .. iters+1 with w = chi (or 1 - chi), and the Rayleigh quotient
lambda = (u, w u)/(u, u) taken at u_{iters+1} (u lies in E, so this equals
(u, Gamma_1 w Gamma_1 u)/(u, u)).
"""
from __future__ import annotations

import numpy as np

from .solver import GammaOperator


def power_lambda(chi, weight_phase: int, iters: int, e0=(1.0, 0.0, 0.0), symbol="rotated"):
    chi = np.asarray(chi)
    d = chi.ndim
    gamma = GammaOperator(chi.shape, symbol)
    w = chi.astype(np.float64) if weight_phase == 1 else 1.0 - chi.astype(np.float64)
    e0 = np.asarray(e0, dtype=np.float64)[:d].reshape((d,) + (1,) * d)
    u = np.broadcast_to(e0.astype(np.complex128), (d,) + chi.shape).copy()
    lam_hist = []
    for _ in range(iters + 1):
        u = gamma(w[None] * u)
        num = float(np.sum(w[None] * np.abs(u) ** 2))
        den = float(np.sum(np.abs(u) ** 2))
        lam_hist.append(num / den)
        u = u / np.sqrt(den)
    return lam_hist[-1], np.array(lam_hist)


def estimate_interval(chi, iters: int = 100, symbol="rotated"):
    """Raw (alpha, beta, mu_min, mu_max) from `iters` power steps on each phase."""
    lam1, _ = power_lambda(chi, 1, iters, symbol=symbol)
    lam2, _ = power_lambda(chi, 0, iters, symbol=symbol)
    mu_max = lam1
    mu_min = 1.0 - lam2
    return 1.0 / mu_max - 1.0, 1.0 / mu_min - 1.0, mu_min, mu_max


def symmetrize(alpha: float, beta: float):
    """Interval with alpha*beta = 1 that contains [alpha, beta]'s inner part.

    Floating-point stability reading: use alpha_u = min(alpha, 1/beta),
    beta_u = 1/alpha_u, so that both zero-weight eigenspaces (mu = 0, 1) map
    inside the convergence disk of the accelerated scheme for every real
    sigma1 > 0.
    """
    a = min(alpha, 1.0 / beta)
    return a, 1.0 / a
