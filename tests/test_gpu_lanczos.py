"""GPU parity of the Lanczos support estimate.

The device and the oracle both run the Lanczos process with full
reorthogonalisation (device: classical Gram-Schmidt twice on the stored
spectra; oracle: modified Gram-Schmidt on real-space fields), the same
process in exact arithmetic, so their coefficients agree to rounding and the
extreme Gauss nodes above the rounding-level weight cut-off agree to 1e-9.
"""
import numpy as np
import pytest

from oracle import lanczos as olanczos
from paper_2001_08289_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2001_08289_amd import scfft  # noqa: E402

CASES = {
    "random48x40": (lambda: inputs.random_phase((48, 40), 0.3, seed=5), (1.0, 0.0)),
    "square64": (lambda: inputs.square_array(64), (1.0, 0.0)),
    "square128_ey": (lambda: inputs.square_array(128), (0.0, 1.0)),
    "cube32": (lambda: inputs.cube_array(32), (1.0, 0.0, 0.0)),
    "random24x20x16": (lambda: inputs.random_phase((24, 20, 16), 0.25, seed=9), (0.0, 0.0, 1.0)),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("symbol", ["rotated", "network"])
def test_lanczos_coefficients_match_oracle(case, symbol):
    make, e0 = CASES[case]
    chi = make()
    ao, bo, n0o = olanczos.lanczos(chi, e0, 12, symbol)
    scfft.release()
    got = scfft.lanczos(chi, e0, steps=12, symbol=symbol)
    k = min(len(ao), len(got["a"]))
    assert k >= min(len(ao), 12)
    assert abs(got["norm0"] - n0o) < 1e-12 * n0o
    assert np.abs(got["a"][:k] - ao[:k]).max() < 1e-10
    kb = min(len(bo), len(got["b"]), k - 1)
    assert np.abs(got["b"][:kb] - bo[:kb]).max() < 1e-10


@pytest.mark.parametrize("case", list(CASES))
def test_lanczos_interval_matches_oracle(case):
    make, e0 = CASES[case]
    chi = make()
    ref = olanczos.interval(chi, e0, 60)
    got = scfft.estimate_interval_lanczos(chi, e0, steps=60)
    # an extreme node that has not converged after 60 steps moves with the
    # rounding of either process (the later Lanczos coefficients are
    # ill-conditioned); each lies within its Ritz residual bound of the
    # spectrum, so the two agree within the sum of the bounds
    ao, bo, n0o, blo = olanczos.lanczos(chi, e0, 60, residual=True)
    gl = scfft.lanczos(chi, e0, steps=60)
    rho = []
    for a, b, n0, bl in ((ao, bo, n0o, blo), (gl["a"], gl["b"], gl["norm0"], gl["b_last"])):
        theta, wts = olanczos.gauss_rule(a, b, n0)
        keep = np.flatnonzero(wts > olanczos.REL_WEIGHT * wts.sum())
        bounds = olanczos.ritz_bounds(a, b, bl)
        rho.append((bounds[keep[0]], bounds[keep[-1]]))
    assert abs(got["mu_min"] - ref[4]) < rho[0][0] + rho[1][0] + 1e-9
    assert abs(got["mu_max"] - ref[5]) < rho[0][1] + rho[1][1] + 1e-9
    assert abs(got["alpha_used"] * got["beta_used"] - 1.0) < 1e-12
    assert got["alpha_used"] <= got["alpha"] + 1e-15


def test_small_weight_extreme_node_on_device():
    """The device keeps an extreme node of relative weight ~1e-10 (a random
    6 x 10 map with e0 turned to nearly cancel the top eigenvalue's weight;
    dense eigen-decomposition of Gamma_1 chi Gamma_1 as the reference)."""
    from oracle import dense
    chi = inputs.random_phase((6, 10), 0.4, seed=4)
    d, m = 2, chi.size
    G = dense.gamma_dense(chi.shape, "rotated")
    X = np.diag(np.tile(chi.ravel().astype(float), d))
    lam, phi = np.linalg.eigh(G @ X @ G)
    ux = phi.conj().T @ (G @ (X @ np.concatenate([np.ones(m), np.zeros(m)])))
    uy = phi.conj().T @ (G @ (X @ np.concatenate([np.zeros(m), np.ones(m)])))
    tot = np.abs(ux) ** 2 + np.abs(uy) ** 2
    top = int(np.flatnonzero(tot > 1e-12 * tot.sum()).max())
    t = np.arctan2(-ux[top].real, uy[top].real) + 1e-4
    got = scfft.estimate_interval_lanczos(chi, (np.cos(t), np.sin(t)), steps=d * m)
    assert abs(got["mu_max"] - lam[top]) < 1e-9


def test_lanczos_laminate_one_point_and_square_support():
    """Laminate with e0 across the layers: one node at 1 - f (the process
    stops after one step).  Square array: support [1/4, 0.7407] at 64^2."""
    f = 0.25
    lam = inputs.laminate(32, 2, fraction=f, axis=0)
    got = scfft.lanczos(lam, (1.0, 0.0), steps=10)
    assert len(got["a"]) == 1 and abs(got["a"][0] - (1 - f)) < 1e-13
    assert abs(got["norm0"] - lam.size * f * (1 - f)) < 1e-9 * lam.size
    iv = scfft.estimate_interval_lanczos(inputs.square_array(64), (1.0, 0.0), steps=60)
    assert abs(iv["mu_min"] - 0.25) < 1e-9 and abs(iv["mu_max"] - 0.7406966456) < 1e-6


def test_lanczos_full_size_2048_and_accelerated_solve_with_its_interval():
    """At 2048^2: the Lanczos interval of the square array, and an accelerated
    solve with the interval it recommends converges and matches eq. J47a."""
    chi = torch.as_tensor(inputs.square_array(2048)).cuda()
    iv = scfft.estimate_interval_lanczos(chi, (1.0, 0.0), steps=60)
    assert abs(iv["mu_min"] - 0.25) < 1e-3 and 0.74 < iv["mu_max"] < 0.7501, iv
    r = scfft.solve(chi, 100.0, (1, 0), "acc_em", alpha=iv["alpha_used"], beta=iv["beta_used"],
                    tol=1e-10, max_iter=200, fields=False, history=False)
    assert r["status"] == 0
    assert abs(r["sigma_star"] - np.sqrt(301 / 103)) < 1e-9
