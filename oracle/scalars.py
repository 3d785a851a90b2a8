"""Scalar parameter maps of the paper (oracle, fp64 complex, test infrastructure).

sigma2 = 1 throughout (section 1: "without loss of generality").
Square roots are numpy's principal branch (Re >= 0).
"""
from __future__ import annotations

import numpy as np


def t_map(sigma1, alpha, beta):
    """Slit map t(sigma1) of eq. J3 / J6: sends [-beta, -alpha] to [-inf, 0], t(1) = 1."""
    s = np.asarray(sigma1, dtype=np.complex128)
    return (s + alpha) * (1.0 + beta) / ((s + beta) * (1.0 + alpha))


def t_map_j23(sigma1, p):
    """Same map written through p as in eq. J23: t = 1 + (s-1)/(p1^2 - p2^2 (s-1))."""
    s = np.asarray(sigma1, dtype=np.complex128)
    p1, p2, _ = p
    return 1.0 + (s - 1.0) / (p1 * p1 - p2 * p2 * (s - 1.0))


def p_from_interval(alpha: float, beta: float) -> np.ndarray:
    """Unit (p^T p = 1, bilinear) vector p realising (alpha, beta) through eq. J24.

    Solving the two relations of eq. J24 for p1^2, p2^2 and using
    p1^2 + p2^2 + p3^2 = 1 (section "The vector subspace collection we
    substitute"):
      p1^2 = (1+alpha)(1+beta)/(beta-alpha),  p2^2 = -(1+alpha)/(beta-alpha),
      p3^2 = -alpha(1+beta)/(beta-alpha).
    p2 and p3 are imaginary for 0 < alpha < beta; the signs are immaterial.
    """
    if not beta > alpha:
        raise ValueError("need beta > alpha")
    w = beta - alpha
    sq = np.array([(1 + alpha) * (1 + beta) / w, -(1 + alpha) / w,
                   -alpha * (1 + beta) / w], dtype=np.complex128)
    return np.sqrt(sq)


def interval_from_p(p):
    """(alpha, beta) from p by eq. J24 as printed."""
    p1, p2, _ = p
    alpha = -1.0 - p1 * p1 / (p2 * p2 - 1.0)
    beta = -1.0 - p1 * p1 / (p2 * p2)
    return alpha, beta


def z_ms(sigma1):
    """Expansion variable of the Moulinec-Suquet scheme, eq. J1: (s-1)/(s+1)."""
    s = np.asarray(sigma1, dtype=np.complex128)
    return (s - 1.0) / (s + 1.0)


def z_sqrt(x):
    """(sqrt(x)-1)/(sqrt(x)+1): eq. J2 with x = sigma1, eq. J4/J46 with x = t."""
    w = np.sqrt(np.asarray(x, dtype=np.complex128))
    return (w - 1.0) / (w + 1.0)


def e2_prime(t, p):
    """E2' of eq. J21 with sigma2 = 1 (E1' = 1)."""
    p1, p2, _ = p
    return (1.0 - t) * p1 * p2 / ((t - 1.0) * p2 * p2 + 1.0)


def j3_prime(t, p):
    """J3' of eq. J26 with sigma2 = 1 (E1' = 1)."""
    p1, p2, p3 = p
    return p1 * p3 * (t - 1.0) / ((t - 1.0) * p2 * p2 + 1.0)


def sigma1_from_t(t, alpha, beta):
    """Inverse of the slit map t(sigma1) of eq. J3 (solve the Moebius map for sigma1)."""
    t = np.asarray(t, dtype=np.complex128)
    # t (s+beta)(1+alpha) = (s+alpha)(1+beta)
    return (alpha * (1 + beta) - t * beta * (1 + alpha)) / (t * (1 + alpha) - (1 + beta))


def sigma1_from_z(z, alpha, beta):
    """sigma1 whose accelerated-scheme variable (eq. J4) equals z: sqrt(t) = (1+z)/(1-z)."""
    z = np.asarray(z, dtype=np.complex128)
    w = (1.0 + z) / (1.0 - z)
    return sigma1_from_t(w * w, alpha, beta)


# ---------------------------------------------------------------- closed forms
def obnosov_square_array(sigma1):
    """Exact sigma* of the periodic square array at 25% (eq. J47a)."""
    s = np.asarray(sigma1, dtype=np.complex128)
    return np.sqrt((1.0 + 3.0 * s) / (3.0 + s))


def hashin_shtrikman(sigma1: float, f: float, d: int):
    """Hashin-Shtrikman bounds (lower, upper) for real sigma1 > 1 = sigma2, isotropic."""
    s1, s2 = float(sigma1), 1.0
    lo = s2 + f * (s1 - s2) * d * s2 / (d * s2 + (1 - f) * (s1 - s2))
    hi = s1 + (1 - f) * (s2 - s1) * d * s1 / (d * s1 + f * (s2 - s1))
    return min(lo, hi), max(lo, hi)


def laminate_means(sigma1, f: float):
    """(harmonic, arithmetic) mean of a laminate with fraction f of sigma1."""
    s = complex(sigma1)
    return 1.0 / (f / s + (1 - f)), f * s + (1 - f)
