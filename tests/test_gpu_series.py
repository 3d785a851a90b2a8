"""GPU parity of the series coefficients of eqs. J5-J7 and their evaluation.

Both sides carry rounding noise in c_k that grows like 3.5^k (the zero-weight
modes at sigma1 = 0 and infinity sit at |z| ~ 1/3 for these intervals), so
coefficients are compared against 1e-13 * 3.5^k in fp64; fp32 is checked
through sigma*(sigma1) at |z| < 0.3, where that noise stays bounded.
"""
import numpy as np
import pytest

from oracle import series as oseries
from oracle import solver as osolver
from paper_2001_08289_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2001_08289_amd import scfft  # noqa: E402


@pytest.mark.parametrize("case", ["square64", "random48x40", "laminate3d", "cube32"])
@pytest.mark.parametrize("symbol", ["rotated", "network"])
def test_series_coefficients_fp64_match_oracle(case, symbol):
    alpha, beta, e0 = 0.25, 4.0, (1.0, 0.0)
    if case == "square64":
        chi = inputs.square_array(64)
    elif case == "random48x40":
        chi = inputs.random_phase((48, 40), 0.3, seed=5)
        alpha, beta = 0.1, 10.0
    elif case == "laminate3d":
        chi = inputs.laminate(16, 3, fraction=0.25, axis=2)
        e0 = (0.0, 0.0, 1.0)
    else:
        chi = inputs.cube_array(32)
        alpha, beta, e0 = 0.19, 5.3, (1.0, 0.0, 0.0)
    n = 16
    ref = oseries.series_coefficients(chi, e0, alpha, beta, n, symbol)
    scfft.release()
    got = scfft.series_coefficients(chi, e0, alpha=alpha, beta=beta, nterms=n, precision="fp64",
                                    symbol=symbol)
    k = np.arange(n + 1)
    bound = 1e-13 * 3.5 ** k * np.maximum(1.0, np.abs(ref))
    assert np.all(np.abs(got - ref) <= bound), np.abs(got - ref) / bound


@pytest.mark.parametrize("precision,bound", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_series_sum_and_pade_match_direct_solves(precision, bound):
    """sigma*(sigma1) from one coefficient run equals the oracle's accelerated
    solve at several sigma1 (partial sum and Pade approximant)."""
    alpha, beta = 0.25, 4.0
    chi = inputs.square_array(128)
    c = scfft.series_coefficients(chi, (1.0, 0.0), alpha=alpha, beta=beta, nterms=48,
                                  precision=precision)
    s1 = np.array([10.0, 100.0, 0.05, 2 + 1j, 1e3])
    ref = np.array([osolver.solve(chi, s, [1, 0], "acc_em", alpha=alpha, beta=beta, tol=1e-14,
                                  max_iter=3000)["sigma_star"] for s in s1])
    got = scfft.series_evaluate(c, s1, alpha=alpha, beta=beta)
    assert np.abs(got - ref).max() < bound * np.abs(ref).max()
    pad = scfft.series_evaluate(c[:25], s1, alpha=alpha, beta=beta, pade_m=12)
    assert np.abs(pad - ref).max() < 10 * bound * np.abs(ref).max()


def test_series_full_size_2048_matches_gpu_solves():
    """At the benchmark size: sigma* from 40 coefficients (fp64) against
    direct accelerated solves on the GPU and against eq. J47a."""
    alpha, beta = 0.25, 4.0
    chi = torch.as_tensor(inputs.square_array(2048)).cuda()
    c = scfft.series_coefficients(chi, (1.0, 0.0), alpha=alpha, beta=beta, nterms=40,
                                  precision="fp64")
    for s in (10.0, 100.0, 0.01):
        direct = scfft.solve(chi, s, (1, 0), "acc_em", alpha=alpha, beta=beta, tol=1e-12,
                             max_iter=500, fields=False, history=False)["sigma_star"]
        ser = scfft.series_evaluate(c, [s], alpha=alpha, beta=beta)[0]
        j47a = np.sqrt((1 + 3 * s) / (3 + s))
        assert abs(ser - direct) < 1e-11 * abs(direct)
        assert abs(ser - j47a) < 1e-11 * j47a
