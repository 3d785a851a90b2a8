"""Own FFT for the oracle (test infrastructure, fp64, numpy).

Unnormalised forward DFT  X[k] = sum_j x[j] exp(-2 pi i j k / n)  and inverse
x[j] = (1/n) sum_k X[k] exp(+2 pi i j k / n), the transforms the FFT methods
use to go back and forth between real and Fourier space (section 1, the
paragraph after eq. J0-0).

Recursive decimation in time: for n = p*m with p the smallest prime factor,
the p interleaved subsequences x[j*p + r] are transformed (length m), twisted
by exp(-2 pi i r k / n) and combined by a p-point DFT.  A prime length is a
direct O(n^2) DFT.  Everything is vectorised over the leading axes.
Pinned against numpy.fft and against a direct DFT in the tests.
"""
from __future__ import annotations

import numpy as np


def _smallest_factor(n: int) -> int:
    p = 2
    while p * p <= n:
        if n % p == 0:
            return p
        p += 1
    return n


def _dft_matrix(p: int, sign: float) -> np.ndarray:
    j = np.arange(p)
    return np.exp(sign * 2j * np.pi * ((np.outer(j, j)) % p) / p)


def _fft_last(x: np.ndarray, sign: float) -> np.ndarray:
    """Unnormalised DFT along the last axis with exponent sign `sign`."""
    n = x.shape[-1]
    if n == 1:
        return x.astype(np.complex128, copy=True)
    p = _smallest_factor(n)
    if p == n:
        # direct DFT: X[k] = sum_j x[j] w^(j k)
        return x @ _dft_matrix(n, sign)
    m = n // p
    lead = x.shape[:-1]
    # sub[..., r, j] = x[..., j*p + r]
    sub = np.ascontiguousarray(np.swapaxes(x.reshape(lead + (m, p)), -1, -2))
    y = _fft_last(sub, sign)                     # y[..., r, k], k < m
    r = np.arange(p)[:, None]
    k = np.arange(m)[None, :]
    y = y * np.exp(sign * 2j * np.pi * ((r * k) % n) / n)
    w = _dft_matrix(p, sign)                     # w[q, r] = exp(sign 2 pi i q r / p)
    out = np.empty(lead + (p, m), dtype=np.complex128)
    for q in range(p):
        acc = w[q, 0] * y[..., 0, :]
        for rr in range(1, p):
            acc = acc + w[q, rr] * y[..., rr, :]
        out[..., q, :] = acc
    # X[k + m*q] lives at out[..., q, k]
    return out.reshape(lead + (n,))


def fft(x: np.ndarray, axis: int = -1) -> np.ndarray:
    """Unnormalised forward DFT along one axis."""
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    return np.moveaxis(_fft_last(x, -1.0), -1, axis)


def ifft(x: np.ndarray, axis: int = -1) -> np.ndarray:
    """Inverse DFT along one axis (includes the 1/n factor)."""
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    n = x.shape[-1]
    return np.moveaxis(_fft_last(x, 1.0) / n, -1, axis)


def fftn(x: np.ndarray, axes) -> np.ndarray:
    out = np.asarray(x, dtype=np.complex128)
    for a in axes:
        out = fft(out, a)
    return out


def ifftn(x: np.ndarray, axes) -> np.ndarray:
    out = np.asarray(x, dtype=np.complex128)
    for a in axes:
        out = ifft(out, a)
    return out
