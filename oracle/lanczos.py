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
from the extreme nodes whose weight is not negligible and which pass the
Cullum-Willoughby test for spurious nodes (needed by a recurrence without
reorthogonalisation; harmless here), and the interval actually used follows the floating-point stability rule of the accelerated
scheme: alpha_u = min(alpha, 1/beta), beta_u = 1/alpha_u.
"""
from __future__ import annotations

import numpy as np

from .solver import GammaOperator


def lanczos(chi, e0, steps: int, symbol="rotated"):
    """Coefficients (a_0..a_{m-1}, b_1..b_{m-1}) and |v_0|^2; m <= steps
    (fewer if the Krylov space closes)."""
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
    return np.array(a), np.array(b), n0


def gauss_rule(a, b, n0: float = 1.0):
    """Nodes and weights of the Gauss rule of the tridiagonal matrix (a, b)."""
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    theta, vec = np.linalg.eigh(T)
    return theta, n0 * vec[0] ** 2


def spurious(a, b, tol: float = 1e-8):
    """Cullum-Willoughby test: a simple eigenvalue of T that is also an
    eigenvalue of T with its first row and column removed (within tol) does
    not belong to the measure of v_0 (it is produced by rounding once the
    Lanczos vectors lose orthogonality); numerically multiple eigenvalues
    are copies of converged ones and are kept."""
    theta, _ = gauss_rule(a, b)
    if len(a) < 2:
        return np.zeros(len(theta), dtype=bool)
    that = np.linalg.eigvalsh(np.diag(a[1:]) + np.diag(b[1:], 1) + np.diag(b[1:], -1))
    out = np.zeros(len(theta), dtype=bool)
    for i, t in enumerate(theta):
        multiple = np.sum(np.abs(theta - t) < 1e-8) >= 2
        out[i] = (not multiple) and np.min(np.abs(that - t)) < tol
    return out


def support_estimate(a, b, n0: float = 1.0, rel_weight: float = 1e-6):
    """(mu_min, mu_max): extreme Gauss nodes that pass the Cullum-Willoughby
    test and whose weight exceeds rel_weight times the total weight."""
    theta, wts = gauss_rule(a, b, n0)
    keep = (wts > rel_weight * wts.sum()) & ~spurious(a, b)
    return float(theta[keep].min()), float(theta[keep].max())


def interval(chi, e0=(1.0, 0.0, 0.0), steps: int = 60, symbol="rotated", rel_weight: float = 1e-6):
    """(alpha, beta, alpha_u, beta_u, mu_min, mu_max)."""
    a, b, n0 = lanczos(chi, e0, steps, symbol)
    mu_min, mu_max = support_estimate(a, b, n0, rel_weight)
    alpha = 1.0 / mu_max - 1.0
    beta = 1.0 / mu_min - 1.0
    alpha_u = min(alpha, 1.0 / beta)
    return alpha, beta, alpha_u, 1.0 / alpha_u, mu_min, mu_max
