"""Python binding of libscfft (argument marshalling only).

Every computation happens in the HIP library; torch provides device memory
and the current stream.  The names follow include/scfft.h.  Importing this
module fails loudly when libscfft.so has not been built.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libscfft.so")

MS, EM, ACC_EM, ACC_MS = 0, 1, 2, 3
SCHEMES = {"ms": MS, "em": EM, "acc_em": ACC_EM, "acc_ms": ACC_MS}
FP64, FP32 = 0, 1
PRECISIONS = {"fp64": FP64, "fp32": FP32}
SYMBOLS = {"rotated": 0, "spectral": 1, "network": 2}

OK, ERR_INVALID_ARG, ERR_SLIT, ERR_NOT_CONVERGED = 0, -1, -2, -3
ERR_DIVERGED, ERR_STAGNATED, ERR_DEVICE, ERR_OOM = -4, -5, -6, -7


class c64(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]

    @staticmethod
    def of(z) -> "c64":
        z = complex(z)
        return c64(z.real, z.imag)

    def value(self) -> complex:
        return complex(self.re, self.im)


class Problem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("n", ctypes.c_int * 3),
                ("phase", ctypes.c_void_p), ("density", ctypes.c_void_p),
                ("sigma1", c64), ("e0", ctypes.c_double * 3)]


class Options(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int), ("precision", ctypes.c_int), ("symbol", ctypes.c_int),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("sigma0_set", ctypes.c_int), ("sigma0", c64),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("check_every", ctypes.c_int), ("stag_window", ctypes.c_int),
                ("div_factor", ctypes.c_double), ("stream", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("E", ctypes.c_void_p), ("J", ctypes.c_void_p), ("sigma_star", c64),
                ("mean_J", c64 * 3), ("iterations", ctypes.c_int), ("residual", ctypes.c_double),
                ("status", ctypes.c_int), ("residual_history", ctypes.c_void_p),
                ("sigma_history", ctypes.c_void_p), ("history_cap", ctypes.c_int),
                ("elapsed_ms", ctypes.c_double)]


EXPORTS = ("scfft_default_options", "scfft_solve", "scfft_solve_noalloc", "scfft_solve_batch",
           "scfft_estimate_interval",
           "scfft_gradient", "scfft_effective_tensor", "scfft_series_coefficients",
           "scfft_series_evaluate", "scfft_lanczos", "scfft_estimate_interval_lanczos",
           "scfft_profile_passes", "scfft_plan_info", "scfft_scheme_scalars", "scfft_sigma1_from_z",
           "scfft_status_string", "scfft_release", "scfft_version")


def load_library(path: str = _LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libscfft.so not built at {path}; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    P, O, R = ctypes.POINTER(Problem), ctypes.POINTER(Options), ctypes.POINTER(Result)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.scfft_default_options.argtypes = [O]
    lib.scfft_default_options.restype = None
    lib.scfft_solve.argtypes = [P, O, R]
    lib.scfft_solve.restype = ctypes.c_int
    lib.scfft_solve_noalloc.argtypes = [P, O, R]
    lib.scfft_solve_noalloc.restype = ctypes.c_int
    lib.scfft_solve_batch.argtypes = [ctypes.c_int, P, O, ctypes.c_int, ctypes.POINTER(c64), R]
    lib.scfft_solve_batch.restype = ctypes.c_int
    lib.scfft_estimate_interval.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                            dp, dp, dp, dp]
    lib.scfft_estimate_interval.restype = ctypes.c_int
    lib.scfft_gradient.argtypes = [P, O, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(c64), R, R]
    lib.scfft_gradient.restype = ctypes.c_int
    lib.scfft_effective_tensor.argtypes = [P, O, ctypes.POINTER(c64), ctypes.POINTER(ctypes.c_int)]
    lib.scfft_effective_tensor.restype = ctypes.c_int
    lib.scfft_series_coefficients.argtypes = [P, O, ctypes.c_int, ctypes.POINTER(c64)]
    lib.scfft_series_coefficients.restype = ctypes.c_int
    lib.scfft_series_evaluate.argtypes = [ctypes.c_int, ctypes.POINTER(c64), ctypes.c_double,
                                          ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(c64), ctypes.POINTER(c64)]
    lib.scfft_series_evaluate.restype = ctypes.c_int
    lib.scfft_lanczos.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, dp, dp, dp,
                                  ctypes.POINTER(ctypes.c_int)]
    lib.scfft_lanczos.restype = ctypes.c_int
    lib.scfft_estimate_interval_lanczos.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                                    ctypes.c_double, dp, dp, dp, dp, dp, dp]
    lib.scfft_estimate_interval_lanczos.restype = ctypes.c_int
    lib.scfft_profile_passes.argtypes = [P, O, ctypes.c_int, dp, ctypes.c_int]
    lib.scfft_profile_passes.restype = ctypes.c_int
    lib.scfft_plan_info.argtypes = [P, O, ctypes.POINTER(ctypes.c_int), ctypes.c_int]
    lib.scfft_plan_info.restype = ctypes.c_int
    lib.scfft_scheme_scalars.argtypes = [ctypes.c_int, c64, ctypes.c_double, ctypes.c_double,
                                         ctypes.POINTER(c64)]
    lib.scfft_scheme_scalars.restype = ctypes.c_int
    lib.scfft_sigma1_from_z.argtypes = [ctypes.c_double, ctypes.c_double, c64]
    lib.scfft_sigma1_from_z.restype = c64
    lib.scfft_status_string.argtypes = [ctypes.c_int]
    lib.scfft_status_string.restype = ctypes.c_char_p
    lib.scfft_release.argtypes = []
    lib.scfft_release.restype = None
    lib.scfft_version.argtypes = []
    lib.scfft_version.restype = ctypes.c_char_p
    return lib


_lib = load_library()


class ScfftError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {_lib.scfft_status_string(status).decode()} ({status})")
        self.status = status


def status_string(status: int) -> str:
    return _lib.scfft_status_string(status).decode()


def release() -> None:
    _lib.scfft_release()


def version() -> str:
    return _lib.scfft_version().decode()


def scheme_scalars(scheme: str, sigma1, alpha: float = 0.25, beta: float = 4.0) -> dict:
    out = (c64 * 8)()
    rc = _lib.scfft_scheme_scalars(SCHEMES[scheme], c64.of(sigma1), alpha, beta, out)
    if rc != OK:
        raise ScfftError(rc, "scheme_scalars")
    v = [o.value() for o in out]
    return {"sigma0": v[0], "t": v[1], "z": v[2], "p": np.array(v[3:6]), "e2p": v[6], "j3p": v[7]}


def sigma1_from_z(alpha: float, beta: float, z) -> complex:
    return _lib.scfft_sigma1_from_z(alpha, beta, c64.of(z)).value()


# ---------------------------------------------------------------- helpers
def _torch():
    import torch
    return torch


def _grid_of(t) -> tuple[int, list[int]]:
    shape = list(t.shape)
    d = len(shape)
    if d not in (2, 3):
        raise ValueError("phase/density must be a 2D or 3D array")
    return d, shape[::-1]   # numpy (n1, n0) -> n = (n0, n1)


def _device_array(x, dtype):
    torch = _torch()
    if isinstance(x, torch.Tensor):
        t = x.to(device="cuda", dtype=dtype)
    else:
        t = torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)
    return t.contiguous()


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_problem(phase=None, density=None, sigma1=1.0, e0=(1.0, 0.0, 0.0)):
    """Returns (Problem, keep-alive tensors)."""
    torch = _torch()
    keep = []
    prob = Problem()
    if density is not None:
        dt = _device_array(density, torch.float64)
        keep.append(dt)
        prob.density = dt.data_ptr()
        d, n = _grid_of(dt)
    else:
        pt = _device_array(phase, torch.uint8)
        keep.append(pt)
        prob.phase = pt.data_ptr()
        d, n = _grid_of(pt)
    prob.d = d
    for i in range(3):
        prob.n[i] = n[i] if i < d else 1
    prob.sigma1 = c64.of(sigma1)
    e = list(e0) + [0.0] * (3 - len(e0))
    for i in range(3):
        prob.e0[i] = float(e[i])
    return prob, keep


def make_options(scheme="acc_em", precision="fp64", symbol="rotated", alpha=0.25, beta=4.0,
                 tol=1e-8, max_iter=1000, check_every=16, stag_window=20, div_factor=1e3,
                 sigma0=None, stream=None) -> Options:
    o = Options()
    _lib.scfft_default_options(ctypes.byref(o))
    o.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.symbol = SYMBOLS[symbol] if isinstance(symbol, str) else int(symbol)
    o.alpha, o.beta = float(alpha), float(beta)
    o.tol, o.max_iter, o.check_every = float(tol), int(max_iter), int(check_every)
    o.stag_window, o.div_factor = int(stag_window), float(div_factor)
    if sigma0 is not None:
        o.sigma0_set = 1
        o.sigma0 = c64.of(sigma0)
    o.stream = _stream_ptr(stream)
    return o


def _result_dict(res: Result, d: int, E=None, J=None, hist_r=None, hist_s=None) -> dict:
    n = res.iterations
    out = {"sigma_star": res.sigma_star.value(),
           "mean_J": np.array([res.mean_J[i].value() for i in range(d)]),
           "iterations": n, "residual": res.residual, "status": res.status,
           "elapsed_ms": res.elapsed_ms, "E": E, "J": J}
    if hist_r is not None:
        k = min(n + 1, len(hist_r))
        out["residual_history"] = hist_r[:k].copy()
        out["sigma_history"] = hist_s[:k, 0] + 1j * hist_s[:k, 1]
    return out


def solve(phase=None, sigma1=1.0, e0=(1.0, 0.0, 0.0), scheme="acc_em", *, density=None,
          precision="fp64", symbol="rotated", alpha=0.25, beta=4.0, tol=1e-8, max_iter=1000,
          check_every=16, stag_window=20, div_factor=1e3, sigma0=None, fields=True,
          history=True, raise_on_error=True, stream=None, noalloc=False) -> dict:
    """Run scfft_solve (scfft_solve_noalloc when noalloc is set).  E and J come
    back as complex128 CUDA tensors (d, *grid)."""
    torch = _torch()
    prob, keep = make_problem(phase, density, sigma1, e0)
    opt = make_options(scheme, precision, symbol, alpha, beta, tol, max_iter, check_every,
                       stag_window, div_factor, sigma0, stream)
    grid = tuple(keep[0].shape)
    d = prob.d
    res = Result()
    E = J = None
    if fields:
        E = torch.empty((d,) + grid, dtype=torch.complex128, device="cuda")
        J = torch.empty_like(E)
        res.E, res.J = E.data_ptr(), J.data_ptr()
    hist_r = hist_s = None
    if history:
        cap = max_iter + 1
        hist_r = np.full(cap, np.nan)
        hist_s = np.zeros((cap, 2))
        res.residual_history = hist_r.ctypes.data
        res.sigma_history = hist_s.ctypes.data
        res.history_cap = cap
    fn = _lib.scfft_solve_noalloc if noalloc else _lib.scfft_solve
    rc = fn(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(res))
    if rc in (ERR_INVALID_ARG, ERR_SLIT, ERR_DEVICE, ERR_OOM) and raise_on_error:
        raise ScfftError(rc, "scfft_solve_noalloc" if noalloc else "scfft_solve")
    return _result_dict(res, d, E, J, hist_r, hist_s)


def solve_batch(phases, sigma1s, e0=(1.0, 0.0, 0.0), scheme="acc_em", *, alphas=None, betas=None,
                precision="fp32", symbol="rotated", tol=1e-6, max_iter=1000, check_every=16,
                stag_window=20, div_factor=1e3, fields=False, stream=None) -> list:
    """scfft_solve_batch over len(phases) structures x sigma1s.shape[1] conductivities."""
    torch = _torch()
    nprob = len(phases)
    s1 = np.asarray(sigma1s, dtype=np.complex128).reshape(nprob, -1)
    nsig = s1.shape[1]
    probs = (Problem * nprob)()
    opts = (Options * nprob)()
    keep = []
    for i, ph in enumerate(phases):
        p, k = make_problem(ph, None, 1.0, e0)
        keep += k
        probs[i] = p
        a = alphas[i] if alphas is not None else 0.25
        b = betas[i] if betas is not None else 4.0
        opts[i] = make_options(scheme, precision, symbol, a, b, tol, max_iter, check_every,
                               stag_window, div_factor, None, stream)
    sig = (c64 * (nprob * nsig))()
    for i in range(nprob):
        for j in range(nsig):
            sig[i * nsig + j] = c64.of(s1[i, j])
    results = (Result * (nprob * nsig))()
    Es = []
    if fields:
        for i in range(nprob):
            grid = tuple(keep[i].shape)
            for j in range(nsig):
                E = torch.empty((probs[i].d,) + grid, dtype=torch.complex128, device="cuda")
                Es.append(E)
                results[i * nsig + j].E = E.data_ptr()
    rc = _lib.scfft_solve_batch(nprob, probs, opts, nsig, sig, results)
    if rc in (ERR_INVALID_ARG, ERR_SLIT, ERR_DEVICE, ERR_OOM):
        raise ScfftError(rc, "scfft_solve_batch")
    out = []
    for i in range(nprob):
        for j in range(nsig):
            r = results[i * nsig + j]
            out.append(_result_dict(r, probs[i].d, Es[i * nsig + j] if fields else None))
    return out


def estimate_interval(phase, iters: int = 100, symbol="rotated", stream=None) -> dict:
    prob, keep = make_problem(phase, None, 1.0, (1.0, 0.0, 0.0))
    a, b, mn, mx = (ctypes.c_double() for _ in range(4))
    rc = _lib.scfft_estimate_interval(ctypes.byref(prob), int(iters), SYMBOLS[symbol],
                                      _stream_ptr(stream), ctypes.byref(a), ctypes.byref(b),
                                      ctypes.byref(mn), ctypes.byref(mx))
    if rc != OK:
        raise ScfftError(rc, "scfft_estimate_interval")
    return {"alpha": a.value, "beta": b.value, "mu_min": mn.value, "mu_max": mx.value}


def gradient(phase=None, sigma1=20.0, e0=(1.0, 0.0, 0.0), *, density=None, precision="fp64",
             symbol="rotated", tol=1e-8, max_iter=2000, check_every=16, stag_window=20,
             div_factor=1e3, sigma0=None, stream=None) -> dict:
    """scfft_gradient: d sigma*/d sigma(x), d sigma*/d rho(x), d sigma*/d sigma1."""
    torch = _torch()
    prob, keep = make_problem(phase, density, sigma1, e0)
    opt = make_options("em", precision, symbol, 0.25, 4.0, tol, max_iter, check_every,
                       stag_window, div_factor, sigma0, stream)
    grid = tuple(keep[0].shape)
    g = torch.empty(grid, dtype=torch.complex128, device="cuda")
    drho = torch.empty_like(g)
    ds1 = c64()
    fwd, adj = Result(), Result()
    E = torch.empty((prob.d,) + grid, dtype=torch.complex128, device="cuda")
    fwd.E = E.data_ptr()
    rc = _lib.scfft_gradient(ctypes.byref(prob), ctypes.byref(opt), ctypes.c_void_p(g.data_ptr()),
                             ctypes.c_void_p(drho.data_ptr()), ctypes.byref(ds1),
                             ctypes.byref(fwd), ctypes.byref(adj))
    if rc in (ERR_INVALID_ARG, ERR_SLIT, ERR_DEVICE, ERR_OOM):
        raise ScfftError(rc, "scfft_gradient")
    return {"status": rc, "g": g, "drho": drho, "dsigma1": ds1.value(),
            "forward": _result_dict(fwd, prob.d, E), "adjoint": _result_dict(adj, prob.d)}


def effective_tensor(phase=None, sigma1=10.0, scheme="acc_em", *, density=None, precision="fp64",
                     symbol="rotated", alpha=0.25, beta=4.0, tol=1e-10, max_iter=1000, check_every=16,
                     stag_window=20, div_factor=1e3, sigma0=None, stream=None) -> dict:
    """scfft_effective_tensor: the d x d effective conductivity (column j: e0 = e_j)."""
    prob, keep = make_problem(phase, density, sigma1, (1.0, 0.0, 0.0))
    opt = make_options(scheme, precision, symbol, alpha, beta, tol, max_iter, check_every,
                       stag_window, div_factor, sigma0, stream)
    d = prob.d
    out = (c64 * (d * d))()
    its = (ctypes.c_int * d)()
    rc = _lib.scfft_effective_tensor(ctypes.byref(prob), ctypes.byref(opt), out, its)
    if rc in (ERR_INVALID_ARG, ERR_SLIT, ERR_DEVICE, ERR_OOM):
        raise ScfftError(rc, "scfft_effective_tensor")
    t = np.array([out[k].value() for k in range(d * d)]).reshape(d, d)
    return {"tensor": t, "iterations": list(its), "status": rc}


def series_coefficients(phase, e0=(1.0, 0.0, 0.0), *, alpha=0.25, beta=4.0, nterms=40,
                        precision="fp64", symbol="rotated", check_every=16, stream=None) -> np.ndarray:
    """scfft_series_coefficients: c_0 .. c_nterms of sigma*/sqrt(t) = sum c_n z^n."""
    prob, keep = make_problem(phase, None, 1.0, e0)
    opt = make_options("acc_em", precision, symbol, alpha, beta, check_every=check_every,
                       stream=stream)
    out = (c64 * (nterms + 1))()
    rc = _lib.scfft_series_coefficients(ctypes.byref(prob), ctypes.byref(opt), int(nterms), out)
    if rc != OK:
        raise ScfftError(rc, "scfft_series_coefficients")
    return np.array([out[k].value() for k in range(nterms + 1)])


def series_evaluate(coeffs, sigma1s, *, alpha=0.25, beta=4.0, pade_m=0) -> np.ndarray:
    """scfft_series_evaluate: sigma*(sigma1) from the coefficients (partial sum, or
    the [L/M] Pade approximant with M = pade_m)."""
    c = np.asarray(coeffs, dtype=np.complex128).ravel()
    s = np.atleast_1d(np.asarray(sigma1s, dtype=np.complex128)).ravel()
    cin = (c64 * len(c))(*[c64(float(v.real), float(v.imag)) for v in c])
    sin = (c64 * len(s))(*[c64(float(v.real), float(v.imag)) for v in s])
    out = (c64 * max(1, len(s)))()
    rc = _lib.scfft_series_evaluate(len(c) - 1, cin, float(alpha), float(beta), int(pade_m),
                                    len(s), sin, out)
    if rc != OK:
        raise ScfftError(rc, "scfft_series_evaluate")
    return np.array([out[k].value() for k in range(len(s))])


def lanczos(phase, e0=(1.0, 0.0, 0.0), *, steps=60, symbol="rotated", stream=None) -> dict:
    """scfft_lanczos: recurrence coefficients a, b and |v_0|^2 (fp64)."""
    prob, keep = make_problem(phase, None, 1.0, e0)
    a = (ctypes.c_double * steps)()
    b = (ctypes.c_double * steps)()
    n0 = ctypes.c_double()
    m = ctypes.c_int()
    rc = _lib.scfft_lanczos(ctypes.byref(prob), int(steps), SYMBOLS[symbol], _stream_ptr(stream), a,
                            b, ctypes.byref(n0), ctypes.byref(m))
    if rc != OK:
        raise ScfftError(rc, "scfft_lanczos")
    return {"a": np.array(a[:m.value]), "b": np.array(b[:max(0, m.value - 1)]),
            "b_last": b[m.value - 1], "norm0": n0.value}


def estimate_interval_lanczos(phase, e0=(1.0, 0.0, 0.0), *, steps=60, symbol="rotated",
                              rel_weight=1e-20, stream=None) -> dict:
    """scfft_estimate_interval_lanczos: raw and stability-symmetrised interval."""
    prob, keep = make_problem(phase, None, 1.0, e0)
    v = [ctypes.c_double() for _ in range(6)]
    rc = _lib.scfft_estimate_interval_lanczos(ctypes.byref(prob), int(steps), SYMBOLS[symbol],
                                              _stream_ptr(stream), float(rel_weight),
                                              *[ctypes.byref(x) for x in v])
    if rc != OK:
        raise ScfftError(rc, "scfft_estimate_interval_lanczos")
    keys = ("alpha", "beta", "alpha_used", "beta_used", "mu_min", "mu_max")
    return {k: x.value for k, x in zip(keys, v)}


PLAN_INFO_KEYS = ("real", "packed", "pitch", "nontemporal", "x_radix", "gamma_radix",
                  "gamma_tile", "y_tile", "tuned", "x_rows", "x_engine", "gamma_engine",
                  "y_engine")


def plan_info(phase=None, sigma1=10.0, e0=(1.0, 0.0, 0.0), scheme="acc_em", *, density=None,
              precision="fp32", symbol="rotated", alpha=0.25, beta=4.0, stream=None) -> dict:
    """scfft_plan_info: the execution choices (tuned or by rule) of a solve."""
    prob, keep = make_problem(phase, density, sigma1, e0)
    opt = make_options(scheme, precision, symbol, alpha, beta, stream=stream)
    info = (ctypes.c_int * len(PLAN_INFO_KEYS))()
    rc = _lib.scfft_plan_info(ctypes.byref(prob), ctypes.byref(opt), info, len(PLAN_INFO_KEYS))
    if rc != OK:
        raise ScfftError(rc, "scfft_plan_info")
    return dict(zip(PLAN_INFO_KEYS, list(info)))


def profile_passes(phase=None, sigma1=10.0, e0=(1.0, 0.0, 0.0), scheme="acc_em", *, density=None,
                   precision="fp32", symbol="rotated", alpha=0.25, beta=4.0, iters=10,
                   stream=None) -> dict:
    prob, keep = make_problem(phase, density, sigma1, e0)
    opt = make_options(scheme, precision, symbol, alpha, beta, stream=stream)
    ms = (ctypes.c_double * 5)()
    rc = _lib.scfft_profile_passes(ctypes.byref(prob), ctypes.byref(opt), int(iters), ms, 5)
    if rc != OK:
        raise ScfftError(rc, "scfft_profile_passes")
    return {"xpass": ms[0], "gamma": ms[1], "y_fwd": ms[2], "y_inv": ms[3], "finalize": ms[4]}


class DensityConductivity:
    """torch.autograd.Function factory: sigma*(rho, sigma1) with adjoint gradients.

    sigma(x) = 1 + (sigma1 - 1) rho(x) on a 2D/3D grid, e0 fixed; the forward
    value is the real part of sigma* (real sigma1), the backward uses the
    library's adjoint solve (scfft_gradient).
    """

    @staticmethod
    def function(e0=(1.0, 0.0, 0.0), precision="fp64", tol=1e-8, max_iter=2000):
        torch = _torch()

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, rho, sigma1):
                out = gradient(density=rho.detach(), sigma1=float(sigma1), e0=e0,
                               precision=precision, tol=tol, max_iter=max_iter)
                ctx.save_for_backward(out["drho"].real.to(rho.dtype),
                                      torch.tensor(out["dsigma1"].real, dtype=torch.float64))
                return torch.tensor(out["forward"]["sigma_star"].real, dtype=torch.float64,
                                    device=rho.device)

            @staticmethod
            def backward(ctx, grad_out):
                drho, ds1 = ctx.saved_tensors
                g = grad_out.to(torch.float64)
                return drho * g.to(drho.device), (ds1.to(g.device) * g)

        return _Fn
