"""Brute-force dense solve of the discrete Lippmann-Schwinger system (oracle).

Eliminating the series of eq. J0-0 gives the linear system
[I + Gamma_1 (sigma/sigma0 - 1)] E = e0 (the isotropic-reference special case
of eq. J47i with Gamma = Gamma_1/sigma0).  Its solution does not depend on
sigma0.  Gamma_1 is assembled as a dense matrix from explicit DFT matrices
(no FFT, no iteration), and the system is solved by LU with partial pivoting
(numpy.linalg.solve).  Only for grids of at most a few hundred voxels.
"""
from __future__ import annotations

import numpy as np

from .solver import local_sigma
from .symbols import symbol_vectors


def _dft_matrix_grid(grid_shape):
    """Unnormalised DFT of a C-ordered flattened grid (numpy shape order)."""
    mat = np.ones((1, 1), dtype=np.complex128)
    for n in grid_shape:
        j = np.arange(n)
        f = np.exp(-2j * np.pi * np.outer(j, j) / n)
        mat = np.kron(mat, f)
    return mat


def gamma_dense(grid_shape, symbol="rotated"):
    """Dense Gamma_1 acting on the stacked vector [E_0; E_1; ...] (component-major)."""
    d = len(grid_shape)
    m = int(np.prod(grid_shape))
    f = _dft_matrix_grid(grid_shape)
    finv = np.conj(f) / m
    vec = symbol_vectors(grid_shape, symbol).reshape(d, m)
    if symbol == "network":
        norm2 = np.sum(np.abs(vec) ** 2, axis=0)
        conjv = np.conj(vec)
    else:
        norm2 = np.sum(vec * vec, axis=0)
        conjv = vec
    safe = np.where(norm2 == 0, 1.0, norm2)
    g = np.zeros((d * m, d * m), dtype=np.complex128)
    for i in range(d):
        for j in range(d):
            sym = np.where(norm2 == 0, 0.0, vec[i] * conjv[j] / safe)
            g[i * m:(i + 1) * m, j * m:(j + 1) * m] = finv @ (sym[:, None] * f)
    return g


def dense_solve(chi, sigma1, e0, symbol="rotated", sigma_field=None, sigma0=None):
    """Exact discrete field E (d, *grid) and sigma* = <sigma E>.e0/|e0|^2."""
    chi = np.asarray(chi)
    grid = chi.shape if sigma_field is None else np.asarray(sigma_field).shape
    d = len(grid)
    m = int(np.prod(grid))
    e0 = np.asarray(e0, dtype=np.float64)[:d]
    sig = local_sigma(chi, sigma1, sigma_field).reshape(m)
    if sigma0 is None:
        sigma0 = (complex(sigma1) + 1.0) / 2.0 if sigma_field is None else complex(np.mean(sig))
    g = gamma_dense(grid, symbol)
    dvec = np.tile(sig / sigma0 - 1.0, d)
    a = np.eye(d * m, dtype=np.complex128) + g * dvec[None, :]
    rhs = np.repeat(e0.astype(np.complex128), m)
    e = np.linalg.solve(a, rhs).reshape((d,) + tuple(grid))
    j = sig.reshape(grid)[None] * e
    mean_j = j.reshape(d, -1).mean(axis=1)
    return {"E": e, "J": j, "mean_J": mean_j,
            "sigma_star": complex(np.dot(mean_j, e0) / np.dot(e0, e0))}


def dense_gradient(chi, sigma1, e0, symbol="rotated", sigma_field=None, h=1e-6):
    """d sigma*/d sigma(x) by central differences of dense solves (tiny grids only)."""
    chi = np.asarray(chi)
    base = local_sigma(chi, sigma1, sigma_field)
    grad = np.zeros(base.shape, dtype=np.complex128)
    for idx in np.ndindex(base.shape):
        sp = base.copy()
        sm = base.copy()
        sp[idx] += h
        sm[idx] -= h
        fp = dense_solve(chi, sigma1, e0, symbol, sigma_field=sp,
                         sigma0=complex(np.mean(base)))["sigma_star"]
        fm = dense_solve(chi, sigma1, e0, symbol, sigma_field=sm,
                         sigma0=complex(np.mean(base)))["sigma_star"]
        grad[idx] = (fp - fm) / (2 * h)
    return grad
