"""Pins of the oracle's scheme iterates against the paper's series.

Each scheme's iterates are partial sums of the expansion of the effective
conductivity in that scheme's variable z (eq. J0-0 / J1 for MS, eq. J2 for
EM, eqs. J42a / J43 for the schemes in H''), because iterate 0 is the source
term and every iteration applies the same linear operator once more:

  MS, MS in H'' (reference sigma0):  <J^n>.e0/|e0|^2 = sigma0 T_{n+1}(z)
  EM, EM in H'' (P = J + sigma0 E):  <J^n>.e0/|e0|^2 = sigma0 [T_n(z) + c_{n+1} z^{n+1}/2]

where f(z) = sigma*/sigma0 = sum_k c_k z^k and T_n is its degree-n Taylor
polynomial.  (MS: <sigma E^n>/sigma0 = <E^n> + z <K E^n> with
sigma/sigma0 = 1 + z K, one power of z beyond E^n.  EM: J = (P + Z P)/2,
<P^n> = 2 sigma0 e0 + <Z P^{n-1}> and Z = z K, so the mean of the last
term enters with weight 1/2.)  In H'' the current is J'' = sigma'' E'' and
its Q-slot mean is compared.

The coefficients c_k come from closed forms, not from any solver: the
harmonic mean of a laminate (exact on every grid and for every symbol) and
eq. J47a for the square array (the discrete sigma* of the 64^2 grid matches
it to ~1e-12), expanded by the Cauchy integral on |z| = 0.6 with sigma1(z),
sigma0(z) written out per scheme.  A dropped term, a wrong sign or a wrong
relaxation in any scheme's update changes some iterate and fails here.
"""
import numpy as np
import pytest

from oracle import solver as osolver
from paper_2001_08289_amd import inputs

ALPHA, BETA = 0.25, 4.0


def _sigma1_from_t(t):
    # t(sigma1) = (sigma1 + alpha)(1 + beta) / ((sigma1 + beta)(1 + alpha))  (eq. J3) inverted
    return (ALPHA * (1 + BETA) - t * BETA * (1 + ALPHA)) / (t * (1 + ALPHA) - (1 + BETA))


# scheme -> (sigma1(z), sigma0(z), z(sigma1))
MAPS = {
    "ms": (lambda z: (1 + z) / (1 - z), lambda z: 1 / (1 - z),
           lambda s: (s - 1) / (s + 1)),
    "em": (lambda z: ((1 + z) / (1 - z)) ** 2, lambda z: (1 + z) / (1 - z),
           lambda s: (np.sqrt(s) - 1) / (np.sqrt(s) + 1)),
    "acc_em": (lambda z: _sigma1_from_t(((1 + z) / (1 - z)) ** 2), lambda z: (1 + z) / (1 - z),
               None),
    "acc_ms": (lambda z: _sigma1_from_t((1 + z) / (1 - z)), lambda z: 1 / (1 - z), None),
}


def _taylor(func, nmax, r=0.6, m=2048):
    """Taylor coefficients of an analytic function by the trapezoid rule on |z| = r."""
    z = r * np.exp(2j * np.pi * (np.arange(m) + 0.5) / m)
    v = func(z)
    return np.array([np.mean(v * z ** (-k)) for k in range(nmax + 1)])


def _square(s1):
    return np.sqrt((1 + 3 * s1) / (3 + s1))   # eq. J47a, principal branch


def _harmonic(s1, f=0.25):
    return 1.0 / (f / s1 + (1 - f))


GEOMS = {
    "laminate_2d": (lambda: inputs.laminate(32, 2, 0.25, axis=0, seed=0), _harmonic, [1.0, 0.0],
                    1e-12),
    "laminate_3d": (lambda: inputs.laminate(8, 3, 0.25, axis=0, seed=0), _harmonic,
                    [1.0, 0.0, 0.0], 1e-12),
    "square_64": (lambda: inputs.square_array(64), _square, [1.0, 0.0], 1e-9),
}


@pytest.mark.parametrize("geom", sorted(GEOMS))
@pytest.mark.parametrize("scheme", sorted(MAPS))
@pytest.mark.parametrize("s1", [10.0, 0.01, 3 + 2j])
def test_iterates_are_partial_sums(geom, scheme, s1):
    make, closed, e0, tol = GEOMS[geom]
    if geom == "laminate_3d" and s1 == 0.01:
        pytest.skip("covered in 2D")
    chi = make()
    s1z, s0z, zof = MAPS[scheme]
    c = _taylor(lambda z: closed(s1z(z)) / s0z(z), 16)
    nmax = 12
    d = len(e0)
    hist = None
    for n in range(nmax + 1):
        if scheme in ("ms", "em"):
            if hist is None:
                r = osolver.solve(chi, s1, e0, scheme, tol=-1, max_iter=nmax, stag_window=0,
                                  div_factor=0)
                hist = r["sigma_history"]
                par = r["params"]
            val = hist[n]
        else:
            r = osolver.solve(chi, s1, e0, scheme, alpha=ALPHA, beta=BETA, tol=-1, max_iter=n,
                              stag_window=0, div_factor=0)
            par = r["params"]
            val = np.dot(r["slots_J"][0].reshape(d, -1).mean(axis=1), e0) / np.dot(e0, e0)
        z = par["z"] if "z" in par else zof(complex(s1))
        s0 = par["sigma0"]
        if scheme in ("ms", "acc_ms"):
            pred = s0 * np.polyval(c[:n + 2][::-1], z)
        else:
            pred = s0 * (np.polyval(c[:n + 1][::-1], z) + 0.5 * c[n + 1] * z ** (n + 1))
        assert abs(val - pred) < tol * abs(pred), (n, val, pred)
