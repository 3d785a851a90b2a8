"""Lanczos estimate of the support of the spectral measure (oracle, fp64).

Test infrastructure: only tests, the smoke check and the benchmark's CPU
baseline use this module.

sigma*(sigma1) is singular where sigma1 = 1 - 1/mu for mu in the support of
the spectral measure of A = Gamma_1 chi Gamma_1 on E with respect to the
start vector v_0 = Gamma_1 chi e0 (the resolvent behind the series of
eq. J0-0).  The paper needs estimates of the interval [-beta, -alpha] that
contains these singularities (section "Estimating the parameters alpha and
beta") and stresses that the support depends on fine details of the
microstructure.  Here the extreme points of the support are estimated by
the Lanczos process on A from v_0 (textbook form, Hermitian inner product,
full reorthogonalisation so that no spurious copies appear):
    q_0 = v_0/|v_0|,  w = A q_j - b_j q_{j-1},  a_j = (q_j, w),
    w <- w - a_j q_j (then reorthogonalised against q_0..q_j),
    b_{j+1} = |w|,  q_{j+1} = w / b_{j+1}.
The eigenvalues theta_i of the tridiagonal matrix T (diagonal a, off-diagonal
b) are the Gauss nodes of the measure; the squared first components of its
eigenvectors, times |v_0|^2, are the Gauss weights.  Then
    alpha = 1/mu_max - 1,   beta = 1/mu_min - 1
from the extreme nodes whose relative weight exceeds rel_weight = 1e-20,
and the interval actually used follows the floating-point stability rule of
the accelerated scheme: alpha_u = min(alpha, 1/beta), beta_u = 1/alpha_u.

The cut-off separates the measure of v_0 from rounding.  With full
reorthogonalisation the Lanczos vectors are orthonormal to fp64 rounding
(eps ~ 1e-16), so a Ritz vector that the measure does not support still
overlaps v_0 by O(eps) and its Gauss weight is O(eps^2) ~ 1e-32 of the total
(such nodes appear once the Krylov space is exhausted, typically at mu ~ 0
and mu ~ 1, the zero-weight eigenspaces of fields supported in one phase).
A node of weight w of the measure itself is resolved as long as w is far
above that level, so the threshold sits at 1e-20, twelve orders above
rounding and below any weight the tests' maps produce (pinned against a
dense eigen-decomposition with an extreme node of relative weight ~1e-10).
"""
from __future__ import annotations

import numpy as np

from .solver import GammaOperator


def lanczos(chi, e0, steps: int, symbol="rotated", residual=False):
    """Coefficients (a_0..a_{m-1}, b_1..b_{m-1}) and |v_0|^2; m <= steps
    (fewer if the Krylov space closes).  With residual=True also b_m, the
    norm of the last residual (0 when the space closed): a Ritz value theta_i
    lies within b_m |s_{m,i}| of an eigenvalue of A (s_i its eigenvector of
    the tridiagonal matrix)."""
    chi = np.asarray(chi)
    d = chi.ndim
    gamma = GammaOperator(chi.shape, symbol)
    w = chi.astype(np.float64)[None]
    e0v = np.asarray(e0, dtype=np.float64)[:d].reshape((d,) + (1,) * d)
    v0 = gamma(w * np.broadcast_to(e0v, (d,) + chi.shape).astype(np.complex128))
    n0 = float(np.vdot(v0, v0).real)
    Qs = [v0 / np.sqrt(n0)]
    a, b = [], []
    for j in range(steps):
        q = Qs[-1]
        r = gamma(w * q)
        if j > 0:
            r = r - b[-1] * Qs[-2]
        aj = float(np.vdot(q, r).real)
        a.append(aj)
        r = r - aj * q
        for qq in Qs:                       # full reorthogonalisation
            r = r - np.vdot(qq, r) * qq
        bj = float(np.sqrt(np.vdot(r, r).real))
        if j == steps - 1 or bj < 1e-12 * max(1.0, abs(aj)):
            break
        b.append(bj)
        Qs.append(r / bj)
    if residual:
        return np.array(a), np.array(b), n0, (bj if j == steps - 1 else 0.0)
    return np.array(a), np.array(b), n0


def ritz_bounds(a, b, b_last):
    """Residual bound b_m |s_{m,i}| of every Gauss node (same order as
    gauss_rule's nodes)."""
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    _, vec = np.linalg.eigh(T)
    return b_last * np.abs(vec[-1])


def gauss_rule(a, b, n0: float = 1.0):
    """Nodes and weights of the Gauss rule of the tridiagonal matrix (a, b)."""
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    theta, vec = np.linalg.eigh(T)
    return theta, n0 * vec[0] ** 2


REL_WEIGHT = 1e-20


def support_estimate(a, b, n0: float = 1.0, rel_weight: float = REL_WEIGHT):
    """(mu_min, mu_max): extreme Gauss nodes whose weight exceeds rel_weight
    times the total weight."""
    theta, wts = gauss_rule(a, b, n0)
    keep = wts > rel_weight * wts.sum()
    return float(theta[keep].min()), float(theta[keep].max())


def interval(chi, e0=(1.0, 0.0, 0.0), steps: int = 60, symbol="rotated",
             rel_weight: float = REL_WEIGHT):
    """(alpha, beta, alpha_u, beta_u, mu_min, mu_max)."""
    a, b, n0 = lanczos(chi, e0, steps, symbol)
    mu_min, mu_max = support_estimate(a, b, n0, rel_weight)
    alpha = 1.0 / mu_max - 1.0
    beta = 1.0 / mu_min - 1.0
    alpha_u = min(alpha, 1.0 / beta)
    return alpha, beta, alpha_u, 1.0 / alpha_u, mu_min, mu_max
