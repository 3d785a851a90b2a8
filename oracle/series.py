"""Series coefficients of sigma*(sigma1) in the accelerated variable (oracle, fp64).

Test infrastructure: only tests, the smoke check and the benchmark's CPU
baseline use this module.

The expansion of eqs. J5 / J7:
    sigma* / sqrt(t) = 1 + sum_{n >= 1} c_n z^n,
    t = t(sigma1) of eq. J6,   z = (sqrt t - 1) / (sqrt t + 1).
The c_n depend on the geometry, e0 and (alpha, beta) only, so one run gives
sigma* for every sigma1 off the slit [-beta, -alpha].

Derivation used (section "Substitution at the level of the Hilbert space"
and eqs. J27-J45): in H'' with sigma0'' = sqrt(t) the Eyre-Milton operator
Z'' = (sigma'' - sigma0'')/(sigma'' + sigma0'') equals z K, where K = 2 p p^T - I
at phase-1 voxels (sigma'' = I + (t - 1) p p^T, p from eq. J24) and K = -1 on
Q at phase-2 voxels; W'' = I - 2 Gamma_1'' maps Q -> (I - 2 Gamma_1) Q,
S -> -S, T -> T (eq. J44).  The fixed point P'' = W'' Z'' P'' + 2 sqrt(t) e0
expands as P'' = 2 sqrt(t) sum_k z^k u_k with
    u_0 = (e0, 0, 0),   u_k = W'' K u_{k-1},
and J'' = (P'' + Z'' P'') / 2.  Because Gamma_1 removes the mean,
<(W'' v)_Q> = <v_Q>, which gives
    c_0 = 1,   c_k = 2 <(K u_{k-1})_Q> . e0 / |e0|^2      (k >= 1).

Pade approximants (the paper's remark after the numerical results): the
[L/M] approximant of f(z) = sum c_n z^n with denominator q (q_0 = 1) solves
sum_{j=0..M} q_j c_{L+i-j} = 0 for i = 1..M, and its numerator is
a_i = sum_{j=0..min(i,M)} q_j c_{i-j}, i = 0..L.
"""
from __future__ import annotations

import numpy as np

from . import scalars
from .solver import GammaOperator


def series_coefficients(chi, e0, alpha: float, beta: float, nterms: int, symbol="rotated"):
    """c_0 .. c_nterms of eq. J7 for the two-phase map chi (1 = phase 1)."""
    chi = np.asarray(chi)
    d = chi.ndim
    gamma = GammaOperator(chi.shape, symbol)
    p = scalars.p_from_interval(alpha, beta)
    ph = chi.astype(bool)[None]
    e0v = np.asarray(e0, dtype=np.float64)[:d]
    Q = np.broadcast_to(e0v.reshape((d,) + (1,) * d).astype(np.complex128),
                        (d,) + chi.shape).copy()
    S = np.zeros_like(Q)
    T = np.zeros_like(Q)
    c = np.zeros(nterms + 1, dtype=np.complex128)
    c[0] = 1.0
    for k in range(1, nterms + 1):
        s = p[0] * Q + p[1] * S + p[2] * T          # p^T (Q, S, T), bilinear
        KQ = np.where(ph, 2.0 * p[0] * s - Q, -Q)
        KS = np.where(ph, 2.0 * p[1] * s - S, 0.0)
        KT = np.where(ph, 2.0 * p[2] * s - T, 0.0)
        mean = KQ.reshape(d, -1).mean(axis=1)
        c[k] = 2.0 * np.dot(mean, e0v) / np.dot(e0v, e0v)
        Q = KQ - 2.0 * gamma(KQ)
        S = -KS
        T = KT
    return c


def z_of_sigma1(sigma1, alpha: float, beta: float):
    """(sqrt t, z) of eqs. J6-J7 (principal square root)."""
    w = np.sqrt(scalars.t_map(sigma1, alpha, beta))
    return w, (w - 1.0) / (w + 1.0)


def evaluate(c, sigma1, alpha: float, beta: float):
    """Partial sum sqrt(t) sum_n c_n z^n at each sigma1."""
    w, z = z_of_sigma1(sigma1, alpha, beta)
    acc = np.zeros_like(np.asarray(z, dtype=np.complex128))
    for cn in np.asarray(c)[::-1]:
        acc = acc * z + cn
    return w * acc


def pade(c, m: int):
    """Numerator a (degree L = len(c) - 1 - m) and denominator q (degree m, q_0 = 1)."""
    c = np.asarray(c, dtype=np.complex128)
    L = len(c) - 1 - m
    if L < 0 or m < 0:
        raise ValueError("need m <= len(c) - 1")

    def cc(i):
        return c[i] if 0 <= i < len(c) else 0.0

    q = np.ones(m + 1, dtype=np.complex128)
    if m > 0:
        A = np.array([[cc(L + i - j) for j in range(1, m + 1)] for i in range(1, m + 1)])
        rhs = -np.array([cc(L + i) for i in range(1, m + 1)])
        q[1:] = np.linalg.solve(A, rhs)
    a = np.array([sum(q[j] * cc(i - j) for j in range(0, min(i, m) + 1)) for i in range(L + 1)])
    return a, q


def evaluate_pade(a, q, sigma1, alpha: float, beta: float):
    """sqrt(t) a(z) / q(z) at each sigma1."""
    w, z = z_of_sigma1(sigma1, alpha, beta)
    num = np.zeros_like(np.asarray(z, dtype=np.complex128))
    den = np.zeros_like(num)
    for an in np.asarray(a)[::-1]:
        num = num * z + an
    for qn in np.asarray(q)[::-1]:
        den = den * z + qn
    return w * num / den
