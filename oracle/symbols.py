"""Discrete Gamma_1 symbol (oracle, fp64, test infrastructure).

The paper's projection onto curl-free zero-mean fields is
Gamma_1 = k (x) k / |k|^2 for k != 0 and 0 at k = 0 (eq. J11, and eq. J45 for
the Q-slot of H'').  The paper is continuum-only; on an N^d voxel grid the
wavevector k is replaced by a discrete vector n(m) per DFT mode m.  Three
readings are provided (theta_j = 2 pi m_j / n_j).  The periodic cell is the
unit square (cube) and a voxel is 1/n_j wide along axis j, so each difference
quotient carries the factor 1/h_j = n_j (on a grid with equal n_j the factor
cancels in Gamma_1):

  rotated   n_j = n_j sin(theta_j/2) prod_{l != j} cos(theta_l/2)  (default;
            the symbol of the difference across a voxel averaged over the
            other axes); modes with n = 0 but m != 0 (two or more Nyquist
            indices) use n_j = n_j [m_j == n_j/2];
  spectral  the literal k of eq. J11 (up to the common factor 2 pi): signed
            integer m_j in (-n/2, n/2]; at a mode with a Nyquist index and
            another non-zero non-Nyquist index the Nyquist components are
            set to 0 (keeps real fields real);
  network   n_j = n_j (exp(i theta_j) - 1) (forward difference of the
            resistor network of section 2), used as n (n^H . )/|n|^2.

Layout: fields are (d, *grid) with grid shaped (n1, n0) or (n2, n1, n0);
vector component c points along grid axis c, which is numpy axis d-1-c.
"""
from __future__ import annotations

import numpy as np

SYMBOLS = ("rotated", "spectral", "network")


def _mode_indices(grid_shape):
    """List m_c (broadcastable int arrays) for c = 0..d-1 and sizes n_c."""
    d = len(grid_shape)
    ms, ns = [], []
    for c in range(d):
        ax = d - 1 - c
        n = grid_shape[ax]
        shape = [1] * d
        shape[ax] = n
        ms.append(np.arange(n).reshape(shape))
        ns.append(n)
    return ms, ns


def symbol_vectors(grid_shape, symbol: str = "rotated") -> np.ndarray:
    """Array (d, *grid) holding n(m) for every mode (complex for 'network')."""
    d = len(grid_shape)
    ms, ns = _mode_indices(grid_shape)
    full = tuple(grid_shape)
    if symbol == "rotated":
        s, c = [], []
        for m, n in zip(ms, ns):
            half = np.pi * m / n                  # theta/2
            sv = np.sin(half)
            cv = np.cos(half)
            sv = np.where(m == 0, 0.0, sv)        # exact zeros of the formulas
            cv = np.where(2 * m == n, 0.0, cv)
            s.append(sv)
            c.append(cv)
        vec = np.zeros((d,) + full)
        for j in range(d):
            v = ns[j] * s[j]
            for l in range(d):
                if l != j:
                    v = v * c[l]
            vec[j] = np.broadcast_to(v, full)
        norm2 = np.sum(vec * vec, axis=0)
        nonzero_mode = np.zeros(full, dtype=bool)
        for m in ms:
            nonzero_mode |= np.broadcast_to(m != 0, full)
        null = (norm2 == 0.0) & nonzero_mode
        if np.any(null):
            for j in range(d):
                nyq = np.broadcast_to(ns[j] * (2 * ms[j] == ns[j]).astype(float), full)
                vec[j] = np.where(null, nyq, vec[j])
        return vec
    if symbol == "spectral":
        signed = []
        nyq = []
        for m, n in zip(ms, ns):
            sm = np.where(2 * m > n, m - n, m).astype(float)
            signed.append(np.broadcast_to(sm, full))
            nyq.append(np.broadcast_to(2 * m == n, full))
        has_nyq = np.zeros(full, dtype=bool)
        has_other = np.zeros(full, dtype=bool)
        for j in range(d):
            has_nyq |= nyq[j]
            has_other |= (signed[j] != 0) & ~nyq[j]
        drop = has_nyq & has_other
        vec = np.zeros((d,) + full)
        for j in range(d):
            vec[j] = np.where(drop & nyq[j], 0.0, signed[j])
        return vec
    if symbol == "network":
        vec = np.zeros((d,) + full, dtype=np.complex128)
        for j, (m, n) in enumerate(zip(ms, ns)):
            vec[j] = np.broadcast_to(n * (np.exp(2j * np.pi * m / n) - 1.0), full)
        return vec
    raise ValueError(f"unknown symbol {symbol!r}")


def apply_gamma_hat(xhat: np.ndarray, vec: np.ndarray, symbol: str = "rotated") -> np.ndarray:
    """Gamma_1 in Fourier space: n (n . xhat)/|n|^2 per mode, 0 at m = 0 (eq. J11)."""
    if symbol == "network":
        dot = np.sum(np.conj(vec) * xhat, axis=0)
        norm2 = np.sum(np.abs(vec) ** 2, axis=0)
    else:
        dot = np.sum(vec * xhat, axis=0)
        norm2 = np.sum(vec * vec, axis=0)
    safe = np.where(norm2 == 0.0, 1.0, norm2)
    coef = np.where(norm2 == 0.0, 0.0, dot / safe)
    return vec * coef[None]
