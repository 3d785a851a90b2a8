"""Gradient of sigma* with respect to the local conductivity (oracle).

For the bilinear pairing, curl-free and divergence-free zero-mean fields are
orthogonal (the decomposition of section 3 with real, even symbols), so
sigma* |e0|^2 = <E . sigma E> is stationary in E and
    d sigma*/d sigma(x) = E(x).E(x) / (N^d |e0|^2)            (closed form).

Adjoint route (what the GPU path computes): the Eyre-Milton fixed point
P = W Z P + 2 sigma0 e0 (W = I - 2 Gamma_1, Z = (sigma-sigma0)/(sigma+sigma0))
with sigma* = c^T P, c = sigma/(sigma+sigma0) e0/(N^d |e0|^2).  The adjoint
variable solves mu = Z W mu + c (the transposed iteration, "Z W" instead of
"W Z"), and with m = N^d |e0|^2 mu and y = W m,
    d sigma*/d sigma(x) = 2 sigma0/(sigma+sigma0)^2 [ y.P + P.e0/2 ] / (N^d |e0|^2).
"""
from __future__ import annotations

import math

import numpy as np

from .solver import GammaOperator, local_sigma, solve


def closed_form(E, e0):
    d = E.shape[0]
    e0 = np.asarray(e0, dtype=np.float64)[:d]
    m = int(np.prod(E.shape[1:]))
    return np.sum(E * E, axis=0) / (m * float(np.dot(e0, e0)))


def adjoint_solve(sig, e0, sigma0, symbol="rotated", tol=1e-10, max_iter=2000,
                  stag_window=20, div_factor=1e3):
    """Iterate y^{n} = W(Z y^{n-1} + c'), y^0 = 0, c' = sigma/(sigma+sigma0) e0.

    y = W m with m = Z y + c' the rescaled adjoint variable.  The residual is
    the relative increment of y (same rule as the forward solvers).
    """
    sig = np.asarray(sig, dtype=np.complex128)
    grid = sig.shape
    d = len(grid)
    gamma = GammaOperator(grid, symbol)
    e0v = np.asarray(e0, dtype=np.float64)[:d]
    e0f = e0v.reshape((d,) + (1,) * d).astype(np.complex128)
    zfac = (sig - sigma0) / (sig + sigma0)
    cfac = sig / (sig + sigma0)
    y = np.zeros((d,) + grid, dtype=np.complex128)
    prev = None
    min_r, since = math.inf, 0
    n, r, status = 0, math.nan, -3
    hist = []
    while True:
        if n >= 1:
            en = float(np.sum(np.abs(y) ** 2))
            r = math.sqrt(float(np.sum(np.abs(y - prev) ** 2)) / en) if en > 0 else math.inf
            hist.append(r)
            if not math.isfinite(r):
                status = -4
                break
            if r <= tol:
                status = 0
                break
            if div_factor > 0 and r > div_factor * min_r:
                status = -4
                break
            if r < min_r:
                min_r, since = r, 0
            else:
                since += 1
            if stag_window > 0 and since >= stag_window:
                status = -5
                break
        else:
            hist.append(math.nan)
        if n >= max_iter:
            break
        prev = y
        mvar = zfac[None] * y + cfac[None] * e0f
        y = mvar - 2.0 * gamma(mvar)
        n += 1
    return {"y": y, "iterations": n, "residual": r, "status": status,
            "residual_history": np.array(hist)}


def adjoint_gradient(E, sig, e0, sigma0, y):
    """d sigma*/d sigma(x) from the forward field E and the adjoint y = W m."""
    d = E.shape[0]
    e0v = np.asarray(e0, dtype=np.float64)[:d]
    m = int(np.prod(E.shape[1:]))
    P = (sig + sigma0)[None] * E
    ydotp = np.sum(y * P, axis=0)
    pdote = np.tensordot(e0v, P, axes=(0, 0))
    return 2.0 * sigma0 / (sig + sigma0) ** 2 * (ydotp + 0.5 * pdote) / (m * float(np.dot(e0v, e0v)))


def density_gradients(rho, sigma1, e0, tol=1e-10, max_iter=2000, symbol="rotated"):
    """sigma* and its derivatives for sigma(x) = 1 + (sigma1 - 1) rho(x).

    Forward: Eyre-Milton with sigma0 = sqrt(sigma_min sigma_max).  Returns
    sigma*, d sigma*/d sigma1 = sum_x g(x) rho(x) and
    d sigma*/d rho(x) = (sigma1 - 1) g(x), with g from the adjoint solve,
    plus g from the closed form for comparison.
    """
    rho = np.asarray(rho, dtype=np.float64)
    sig = local_sigma(None, sigma1, 1.0 + (complex(sigma1) - 1.0) * rho)
    fwd = solve(None, sigma1, e0, "em", symbol=symbol, tol=tol, max_iter=max_iter,
                sigma_field=sig)
    s0 = fwd["params"]["sigma0"]
    adj = adjoint_solve(sig, e0, s0, symbol=symbol, tol=tol, max_iter=max_iter)
    g = adjoint_gradient(fwd["E"], sig, e0, s0, adj["y"])
    return {"sigma_star": fwd["sigma_star"], "g": g,
            "g_closed": closed_form(fwd["E"], e0),
            "dsigma1": complex(np.sum(g * rho)),
            "drho": (complex(sigma1) - 1.0) * g,
            "forward": fwd, "adjoint": adj}
