"""Pins of the discrete Gamma_1 symbols against real-space difference operators.

Each symbol reading of eq. J11 on a grid is the Fourier symbol of a
real-space difference operator D = (D_0, .., D_{d-1}) on the periodic unit
cell (voxel width 1/n_j along axis j).  The discrete problem of
eqs. J12-J13 then reads: find a potential phi with
sum_j D_j^T sigma (e0_j + D_j phi) = 0 (E = e0 + D phi curl free in the
operator's sense, J = sigma E divergence free in the transposed sense), and
sigma* = <J>.e0/|e0|^2.  These tests assemble D directly in real space --
shifts of the grid, no FFT and no symbol table -- solve that system
densely, and compare the field and sigma* with the oracle's Fourier-space
solvers.  A wrong difference convention (backward instead of forward, a
missing conjugation, a missing 1/h_j on a non-square grid) fails them.

  network   D_j = n_j (S_j - I), the forward difference of the resistor
            network of section 2 (edge (x, x + e_j) carries voxel x's
            conductivity; the node balance is D^T J = 0);
  rotated   D_j = n_j (S_j - I) prod_{l != j} (I + S_l)/2, the difference
            across a voxel averaged over the other axes; on grids of odd
            sizes it has no null modes besides the constants, so it fixes
            the oracle's rotated symbol exactly;
  spectral  D_j = the Fourier differentiation matrix along axis j (textbook
            closed form for an odd number of points: entries
            (-1)^(i-k)/(2 sin(pi (i-k)/n)), times 2 pi for the unit cell).

S_j is the periodic shift (S_j phi)(x) = phi(x + e_j).
"""
import numpy as np
import pytest

from oracle import dense as odense
from oracle import solver as osolver
from paper_2001_08289_amd import inputs


def _shift(grid, c, k):
    d = len(grid)
    m = int(np.prod(grid))
    idx = np.arange(m).reshape(grid)
    tgt = np.roll(idx, -k, axis=d - 1 - c).reshape(m)
    s = np.zeros((m, m))
    s[np.arange(m), tgt] = 1.0
    return s


def _fourier_diff(n):
    """Derivative on n equispaced points of the unit interval (n odd)."""
    assert n % 2 == 1
    i = np.arange(n)[:, None]
    k = np.arange(n)[None, :]
    with np.errstate(divide="ignore"):
        dm = np.where(i == k, 0.0, 0.5 * (-1.0) ** ((i - k) % 2) / np.sin(np.pi * (i - k) / n))
    return 2.0 * np.pi * dm


def _operators(grid, symbol):
    d = len(grid)
    m = int(np.prod(grid))
    eye = np.eye(m)
    ops = []
    for c in range(d):
        n = grid[d - 1 - c]
        if symbol == "network":
            ops.append(n * (_shift(grid, c, 1) - eye))
        elif symbol == "rotated":
            op = n * (_shift(grid, c, 1) - eye)
            for l in range(d):
                if l != c:
                    op = op @ (0.5 * (eye + _shift(grid, l, 1)))
            ops.append(op)
        else:
            mats = [np.eye(g) for g in grid]
            mats[d - 1 - c] = _fourier_diff(n)
            op = mats[0]
            for mat in mats[1:]:
                op = np.kron(op, mat)
            ops.append(op)
    return ops


def _direct_solve(chi, s1, e0, symbol):
    grid = chi.shape
    d = len(grid)
    m = chi.size
    sig = (1.0 + (complex(s1) - 1.0) * chi.astype(float)).reshape(m)
    ops = _operators(grid, symbol)
    a = sum(op.T @ (sig[:, None] * op) for op in ops)
    b = -sum(op.T @ (sig * e0[c]) for c, op in enumerate(ops))
    phi = np.linalg.lstsq(a, b, rcond=None)[0]   # defined up to a constant
    e = np.stack([e0[c] + ops[c] @ phi for c in range(d)]).reshape((d,) + grid)
    mean_j = (sig.reshape(grid)[None] * e).reshape(d, -1).mean(axis=1)
    return e, complex(np.dot(mean_j, e0) / np.dot(e0, e0))


def test_fourier_differentiation_matrix_is_spectral():
    n = 9
    x = np.arange(n) / n
    for k in (1, 2, 4):
        assert np.allclose(_fourier_diff(n) @ np.sin(2 * np.pi * k * x),
                           2 * np.pi * k * np.cos(2 * np.pi * k * x), atol=1e-12)


CASES = [("network", (4, 6)), ("network", (6, 4)), ("network", (3, 4, 5)),
         ("rotated", (5, 7)), ("rotated", (9, 5)), ("rotated", (3, 5, 7)),
         ("spectral", (5, 7)), ("spectral", (9, 5)), ("spectral", (3, 5, 7))]


@pytest.mark.parametrize("symbol,shape", CASES)
@pytest.mark.parametrize("s1", [7.0, 3 + 2j, -0.4 + 0.3j])
def test_symbol_is_the_difference_operator(symbol, shape, s1):
    chi = inputs.random_phase(shape, 0.35, seed=3)
    d = len(shape)
    e0 = np.zeros(d)
    e0[0], e0[-1] = 1.0, 0.5
    e_direct, s_direct = _direct_solve(chi, s1, e0, symbol)
    ref = odense.dense_solve(chi, s1, e0, symbol=symbol)
    assert np.abs(ref["E"] - e_direct).max() < 1e-12 * np.abs(e_direct).max()
    assert abs(ref["sigma_star"] - s_direct) < 1e-13 * abs(s_direct)
    it = osolver.solve(chi, s1, e0, "acc_em", alpha=0.02, beta=50.0, symbol=symbol, tol=1e-13,
                       max_iter=5000)
    assert it["status"] == 0
    assert np.abs(it["E"] - e_direct).max() < 1e-10 * np.abs(e_direct).max()


def _disk(n0, n1, r=0.3):
    x = (np.arange(n0) + 0.5) / n0
    y = (np.arange(n1) + 0.5) / n1
    xx, yy = np.meshgrid(x, y)
    return (((xx - 0.5) ** 2 + (yy - 0.5) ** 2) < r * r).astype(np.uint8)


def _tensor_diag(chi, symbol):
    out = []
    for e0 in ([1.0, 0.0], [0.0, 1.0]):
        r = osolver.solve(chi, 10.0, e0, "acc_em", alpha=0.05, beta=20.0, symbol=symbol,
                          tol=1e-11, max_iter=3000)
        assert r["status"] == 0
        out.append(r["sigma_star"].real)
    return np.array(out)


def test_non_square_cell_convention():
    """A disk of radius 0.3 in the unit cell sampled on 64 x 32 voxels (each
    twice as tall as wide) and on 64 x 64: every symbol describes the same
    physical cell, so all of them agree within the discretisation error
    (about 1% here), and exchanging the two axes exchanges sigma*_xx and
    sigma*_yy exactly.  Treating voxels as squares instead (a 64 x 32 cell)
    moves the rotated and network values by about 6%."""
    ref = _tensor_diag(_disk(64, 64), "spectral")
    for symbol in ("rotated", "spectral", "network"):
        wide = _tensor_diag(_disk(64, 32), symbol)
        tall = _tensor_diag(_disk(32, 64), symbol)
        assert np.abs(wide - ref).max() < 0.02 * ref.max(), (symbol, wide, ref)
        assert np.abs(wide - tall[::-1]).max() < 1e-12 * wide.max()
