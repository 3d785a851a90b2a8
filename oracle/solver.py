"""Reference FFT fixed-point solvers (oracle, fp64, test infrastructure).

Problem (eqs. J12-J13): find E in U+E and J in U+J with
J = [(sigma1 - 1) chi + 1] E, <E> = e0; sigma* is defined by <J> = sigma* <E>
(a scalar for square/cubic symmetry).  Here it is reported as
sigma* = <J>.e0/|e0|^2 (bilinear dot, real e0), with <J> also returned.

Four schemes, each written from the paper and the orthogonal decomposition
H = U + E + J of section 3 (Gamma_1 = projection on E, eq. J11):

  ms      Moulinec-Suquet, eq. J0-0: E^{n+1} = e0 + Gamma_1[(1 - sigma/sigma0) E^n],
          sigma0 = (sigma1+1)/2 (paragraph before eq. J1).
  em      Eyre-Milton, the scheme behind eq. J2, sigma0 = sqrt(sigma1).  With
          P = J + sigma0 E and R = J - sigma0 E the orthogonal decomposition
          gives R = (I - 2 Gamma_1) P - 2 sigma0 e0, and locally
          R = Z P, Z = (sigma - sigma0)/(sigma + sigma0); hence the fixed
          point P = (I - 2 Gamma_1)(Z P) + 2 sigma0 e0 and E = P/(sigma+sigma0).
  acc_em  the same Eyre-Milton scheme in the substituted space H'' (eqs. J27-J45,
          expansion eq. J43): fields (Q, chi S, chi T), chi'' = (p p^T) chi,
          sigma'' = I + (t-1) chi'', sigma0'' = sqrt(t), and
          Gamma_1'' : Q -> Gamma_1 Q, S -> S, T -> 0 (eq. J44).
  acc_ms  the Moulinec-Suquet scheme in H'' (expansion eq. J42a),
          sigma0'' = (t+1)/2; the T-slot of E'' stays 0.

Iterate 0 is the source term (E = e0; P = 2 sigma0 e0; Q = 2 sqrt(t) e0), so
iterates are the partial sums of the paper's series.  After every iterate n
the physical field E^n (the Q-slot in H''), <sigma E^n> and, for n >= 1, the
relative increment r_n = ||E^n - E^{n-1}|| / ||E^n|| are formed (the paper
defines no residual; this is the reading used throughout the project).
"""
from __future__ import annotations

import math

import numpy as np

from . import scalars
from .fft import fftn, ifftn
from .symbols import apply_gamma_hat, symbol_vectors

SCHEMES = ("ms", "em", "acc_em", "acc_ms")

STATUS_OK = 0
STATUS_INVALID_ARG = -1
STATUS_SLIT = -2
STATUS_NOT_CONVERGED = -3
STATUS_DIVERGED = -4
STATUS_STAGNATED = -5


class SolverArgError(ValueError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


class GammaOperator:
    """Gamma_1 on (d, *grid) real-space fields: FFT, per-mode symbol, inverse FFT.

    fft = "own" uses the oracle's own FFT (pinned against numpy.fft and a
    direct DFT); fft = "numpy" calls numpy.fft as a library step, for grids
    (256^3) where the own FFT would take minutes.
    """

    def __init__(self, grid_shape, symbol="rotated", fft="own"):
        self.grid_shape = tuple(grid_shape)
        self.d = len(grid_shape)
        self.symbol = symbol
        self.vec = symbol_vectors(grid_shape, symbol)
        self.axes = tuple(range(1, self.d + 1))
        if fft not in ("own", "numpy"):
            raise ValueError(f"unknown fft {fft!r}")
        self.fft = fft

    def __call__(self, x):
        if self.fft == "numpy":
            xh = np.fft.fftn(x, axes=self.axes)
            return np.fft.ifftn(apply_gamma_hat(xh, self.vec, self.symbol), axes=self.axes)
        xh = fftn(x, self.axes)
        return ifftn(apply_gamma_hat(xh, self.vec, self.symbol), self.axes)


def local_sigma(chi, sigma1, sigma_field=None):
    if sigma_field is not None:
        return np.asarray(sigma_field, dtype=np.complex128)
    return 1.0 + (complex(sigma1) - 1.0) * np.asarray(chi, dtype=np.float64)


def scheme_params(scheme, sigma1, alpha=None, beta=None, sigma_field=None, sigma0=None):
    """Scheme scalars (reference conductivities, p, t, z) with the slit checks."""
    s1 = complex(sigma1)
    out = {"scheme": scheme}
    if scheme in ("acc_em", "acc_ms"):
        if sigma_field is not None:
            raise SolverArgError(STATUS_INVALID_ARG, "H'' schemes need a two-phase map")
        if alpha is None or beta is None or not (0.0 < alpha < beta) or not math.isfinite(beta):
            raise SolverArgError(STATUS_INVALID_ARG, "need 0 < alpha < beta < inf")
        if s1.imag == 0.0 and -beta <= s1.real <= -alpha:
            raise SolverArgError(STATUS_SLIT, "sigma1 on the slit [-beta, -alpha]")
        p = scalars.p_from_interval(alpha, beta)
        t = complex(scalars.t_map(s1, alpha, beta))
        w = complex(np.sqrt(t))
        out.update(p=p, t=t, w=w)
        if scheme == "acc_em":
            out["sigma0"] = w
            out["z"] = (w - 1.0) / (w + 1.0)
        else:
            out["sigma0"] = (t + 1.0) / 2.0
            out["z"] = (t - 1.0) / (t + 1.0)
        return out
    if scheme == "ms":
        if sigma0 is None:
            if sigma_field is not None:
                sf = np.asarray(sigma_field).real
                sigma0 = 0.5 * (float(sf.min()) + float(sf.max()))
            else:
                sigma0 = (s1 + 1.0) / 2.0
        if sigma0 == 0:
            raise SolverArgError(STATUS_INVALID_ARG, "sigma0 = 0")
        out["sigma0"] = complex(sigma0)
        return out
    if scheme == "em":
        if sigma0 is None:
            if sigma_field is not None:
                sf = np.asarray(sigma_field).real
                sigma0 = math.sqrt(float(sf.min()) * float(sf.max()))
            else:
                if s1.imag == 0.0 and s1.real <= 0.0:
                    raise SolverArgError(STATUS_SLIT, "Eyre-Milton needs sigma1 off (-inf, 0]")
                sigma0 = np.sqrt(s1)
        out["sigma0"] = complex(sigma0)
        return out
    raise SolverArgError(STATUS_INVALID_ARG, f"unknown scheme {scheme!r}")


def _mean(x, d):
    return x.reshape(x.shape[0], -1).mean(axis=1)


def solve(chi, sigma1, e0, scheme="ms", alpha=None, beta=None, symbol="rotated",
          tol=1e-8, max_iter=500, sigma_field=None, sigma0=None,
          stag_window=20, div_factor=1e3, fft="own"):
    """Run one scheme to tolerance (or exactly max_iter iterates when tol < 0).

    Returns a dict with E, J (d, *grid), sigma_star, mean_J, iterations,
    residual, status, the histories and, for the H'' schemes, the slots of
    E'' and J'' (used by the embedding checks of eqs. J39-J40).
    stag_window = 0 disables the stagnation stop, div_factor = 0 the
    divergence stop.  fft selects the transform (see GammaOperator).
    """
    chi = np.asarray(chi)
    grid = chi.shape if sigma_field is None else np.asarray(sigma_field).shape
    d = len(grid)
    e0 = np.asarray(e0, dtype=np.float64)[:d]
    if d not in (2, 3) or not np.any(e0 != 0):
        raise SolverArgError(STATUS_INVALID_ARG, "bad dimension or zero e0")
    par = scheme_params(scheme, sigma1, alpha, beta, sigma_field, sigma0)
    sig = local_sigma(chi, sigma1, sigma_field)
    gamma = GammaOperator(grid, symbol, fft)
    e0f = e0.reshape((d,) + (1,) * d).astype(np.complex128)
    e0n2 = float(np.dot(e0, e0))
    ch = np.broadcast_to(chi.astype(np.float64), grid) if sigma_field is None else None
    s0 = par["sigma0"]
    shape = (d,) + tuple(grid)

    if scheme == "ms":
        mfac = 1.0 - sig / s0
        state = {"E": np.broadcast_to(e0f, shape).copy()}

        def phys(st):
            return st["E"]

        def step(st):
            return {"E": e0f + gamma(mfac[None] * st["E"])}
    elif scheme == "em":
        zfac = (sig - s0) / (sig + s0)
        state = {"P": np.broadcast_to(2.0 * s0 * e0f, shape).copy()}

        def phys(st):
            return st["P"] / (sig + s0)[None]

        def step(st):
            r = zfac[None] * st["P"]
            return {"P": r - 2.0 * gamma(r) + 2.0 * s0 * e0f}
    elif scheme == "acc_em":
        p1, p2, p3 = par["p"]
        t, w, z = par["t"], par["w"], par["z"]
        kap = 1.0 / (t + w) - 1.0 / (1.0 + w)
        state = {"Q": np.broadcast_to(2.0 * w * e0f, shape).copy(),
                 "S": np.zeros(shape, np.complex128), "T": np.zeros(shape, np.complex128)}

        def phys(st):
            s = p1 * st["Q"] + p2 * st["S"] + p3 * st["T"]
            return st["Q"] / (1.0 + w) + ch[None] * (p1 * kap) * s

        def step(st):
            q, s_, t_ = st["Q"], st["S"], st["T"]
            s = p1 * q + p2 * s_ + p3 * t_
            # Z'' = z (2 p p^T - I) in phase 1, -z on Q in phase 2
            rq = np.where(ch[None] > 0, z * (2.0 * p1 * s - q), -z * q)
            rs = ch[None] * z * (2.0 * p2 * s - s_)
            rt = ch[None] * z * (2.0 * p3 * s - t_)
            # W'' = I - 2 Gamma_1'': Q -> (I - 2 Gamma_1) Q, S -> -S, T -> T (eq. J44)
            return {"Q": rq - 2.0 * gamma(rq) + 2.0 * w * e0f, "S": -rs, "T": rt}
    elif scheme == "acc_ms":
        p1, p2, p3 = par["p"]
        zm = par["z"]
        state = {"E": np.broadcast_to(e0f, shape).copy(), "S": np.zeros(shape, np.complex128)}

        def phys(st):
            return st["E"]

        def step(st):
            eq, es = st["E"], st["S"]
            s = p1 * eq + p2 * es              # E_T = 0
            # I - sigma''/sigma0'' = z_M (I - 2 p p^T) in phase 1, z_M in phase 2
            xq = np.where(ch[None] > 0, zm * (eq - 2.0 * p1 * s), zm * eq)
            xs = ch[None] * zm * (es - 2.0 * p2 * s)
            return {"E": e0f + gamma(xq), "S": xs}
    else:  # pragma: no cover - scheme_params already rejected it
        raise SolverArgError(STATUS_INVALID_ARG, scheme)

    res_hist, sig_hist = [], []
    prev = None
    min_r = math.inf
    since_min = 0
    status = STATUS_NOT_CONVERGED
    n = 0
    r = math.nan
    while True:
        E = phys(state)
        J = sig[None] * E
        mean_j = _mean(J, d)
        sstar = complex(np.dot(mean_j, e0) / e0n2)
        if n >= 1:
            dn = float(np.sum(np.abs(E - prev) ** 2))
            en = float(np.sum(np.abs(E) ** 2))
            r = math.sqrt(dn / en) if en > 0 else math.inf
        res_hist.append(r)
        sig_hist.append(sstar)
        if n >= 1:
            if not (math.isfinite(r) and np.isfinite(sstar)):
                status = STATUS_DIVERGED
                break
            if r <= tol:
                status = STATUS_OK
                break
            if div_factor > 0 and r > div_factor * min_r:
                status = STATUS_DIVERGED
                break
            if r < min_r:
                min_r, since_min = r, 0
            else:
                since_min += 1
            if stag_window > 0 and since_min >= stag_window:
                status = STATUS_STAGNATED
                break
        if n >= max_iter:
            status = STATUS_NOT_CONVERGED
            break
        prev = E
        state = step(state)
        n += 1

    out = {"E": E, "J": J, "sigma_star": sstar, "mean_J": mean_j, "iterations": n,
           "residual": r, "status": status, "residual_history": np.array(res_hist),
           "sigma_history": np.array(sig_hist), "params": par, "state": state}
    if scheme == "acc_em":
        p1, p2, p3 = par["p"]
        t, w = par["t"], par["w"]
        kap = 1.0 / (t + w) - 1.0 / (1.0 + w)
        s = p1 * state["Q"] + p2 * state["S"] + p3 * state["T"]
        es = ch[None] * (state["S"] / (1.0 + w) + p2 * kap * s)
        et = ch[None] * (state["T"] / (1.0 + w) + p3 * kap * s)
        se = p1 * E + p2 * es + p3 * et
        out["slots_E"] = (E, es, et)
        out["slots_J"] = (E + ch[None] * (t - 1.0) * p1 * se,
                          ch[None] * (es + (t - 1.0) * p2 * se),
                          ch[None] * (et + (t - 1.0) * p3 * se))
    elif scheme == "acc_ms":
        # E'' = (E_Q, chi E_S, 0) and J'' = sigma'' E'' with
        # sigma'' = I + (t - 1) chi p p^T (eq. J37)
        p1, p2, p3 = par["p"]
        t = par["t"]
        es = ch[None] * state["S"]
        se = p1 * E + p2 * es
        out["slots_E"] = (E, es, np.zeros_like(E))
        out["slots_J"] = (E + ch[None] * (t - 1.0) * p1 * se,
                          ch[None] * (es + (t - 1.0) * p2 * se),
                          ch[None] * (t - 1.0) * p3 * se)
    return out
