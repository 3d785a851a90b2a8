"""GPU parity on cases the basic parity suite does not reach.

* the 256^3 kernels (real-field x pass with nontemporal streams, row pitch
  padded to cache lines, 256-point y and z passes) on a fully 3D random map,
  every field value after one accelerated iteration, fp64 and fp32;
* real sigma1 (the half-spectrum path) under the spectral and network
  symbols, with kx = 0 and kx = n0/2 packed into one column and without;
* negative real sigma1 off the slit, where the accelerated scheme's
  variable stays inside the unit disk (eqs. J3-J5);
* sigma1 = 0, the paper's convergence case (EM undefined there);
* the divergence stop and a non-finite medium.
"""
import numpy as np
import pytest

from oracle import solver as osolver
from paper_2001_08289_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2001_08289_amd import scfft  # noqa: E402


def _err(got, ref):
    e = got["E"].cpu().numpy()
    return np.abs(e - ref["E"]).max() / np.abs(ref["E"]).max()


def test_full_size_256_cube_one_iteration_matches_oracle():
    chi = inputs.random_phase((256, 256, 256), 0.3, seed=9)
    ref = osolver.solve(chi, 100.0, [1, 0, 0], "acc_em", alpha=0.25, beta=4.0, tol=-1,
                        max_iter=1, stag_window=0, div_factor=0, fft="numpy")
    for precision, bound in (("fp64", 1e-11), ("fp32", 2e-6)):
        got = scfft.solve(chi, 100.0, (1, 0, 0), "acc_em", precision=precision, tol=-1, max_iter=1,
                          stag_window=0, div_factor=0, history=False)
        err = _err(got, ref)
        print(f"256^3 {precision}: field error {err:.2e}", flush=True)
        assert err < bound, (precision, err)
        assert abs(got["sigma_star"] - ref["sigma_star"]) < bound * abs(ref["sigma_star"])
        del got
        torch.cuda.empty_cache()


@pytest.mark.parametrize("pack", ["0", "1"])
@pytest.mark.parametrize("symbol", ["spectral", "network", "rotated"])
@pytest.mark.parametrize("scheme", ["ms", "em", "acc_em"])
def test_real_field_symbols(pack, symbol, scheme, monkeypatch):
    monkeypatch.setenv("SCFFT_PACK", pack)
    scfft.release()
    try:
        for shape in ((64, 128), (48, 32)):
            chi = inputs.random_phase(shape, 0.3, seed=4)
            ref = osolver.solve(chi, 10.0, [1, 0], scheme, alpha=0.25, beta=4.0, symbol=symbol,
                                tol=-1, max_iter=5, stag_window=0, div_factor=0)
            for precision, bound in (("fp64", 1e-11), ("fp32", 2e-6)):
                got = scfft.solve(chi, 10.0, (1, 0), scheme, precision=precision, symbol=symbol,
                                  tol=-1, max_iter=5, stag_window=0, div_factor=0)
                assert _err(got, ref) < bound, (shape, precision)
    finally:
        scfft.release()


@pytest.mark.parametrize("s1", [-10.0, -0.1, 0.0])
@pytest.mark.parametrize("scheme", ["acc_em", "acc_ms", "ms"])
def test_negative_and_zero_sigma1(s1, scheme):
    chi = inputs.square_array(64)
    ref = osolver.solve(chi, s1, [1, 0], scheme, alpha=0.25, beta=4.0, tol=1e-10, max_iter=500)
    got = scfft.solve(chi, s1, (1, 0), scheme, alpha=0.25, beta=4.0, tol=1e-10, max_iter=500)
    assert got["status"] == ref["status"] == 0
    assert got["iterations"] == ref["iterations"]
    assert abs(got["sigma_star"] - ref["sigma_star"]) < 1e-12 * abs(ref["sigma_star"])
    exact = np.sqrt((1 + 3 * s1) / (3 + s1))   # eq. J47a
    assert abs(got["sigma_star"] - exact) < 1e-9 * abs(exact)
    fixed = osolver.solve(chi, s1, [1, 0], scheme, alpha=0.25, beta=4.0, tol=-1, max_iter=6,
                          stag_window=0, div_factor=0)
    got = scfft.solve(chi, s1, (1, 0), scheme, alpha=0.25, beta=4.0, tol=-1, max_iter=6,
                      stag_window=0, div_factor=0)
    assert _err(got, fixed) < 1e-11


def test_em_rejects_sigma1_zero():
    with pytest.raises(scfft.ScfftError) as e:
        scfft.solve(inputs.square_array(32), 0.0, (1, 0), "em")
    assert e.value.status == scfft.ERR_SLIT


@pytest.mark.parametrize("interval,s1,how", [((1.0, 2.0), 100.0, "growth"),
                                            ((2.0, 3.0), 10.0, "overflow")])
def test_divergence_stop_on_device(interval, s1, how):
    """An interval that misses part of the spectrum makes the accelerated
    iterates grow: first the residual climbs past 1e3 times its minimum
    (growth), or, where it never falls far, the fields overflow."""
    chi = inputs.square_array(32)
    a, b = interval
    ref = osolver.solve(chi, s1, [1, 0], "acc_em", alpha=a, beta=b, tol=1e-12, max_iter=3000,
                        stag_window=0)
    got = scfft.solve(chi, s1, (1, 0), "acc_em", alpha=a, beta=b, tol=1e-12, max_iter=3000,
                      stag_window=0, check_every=8, fields=False)
    assert ref["status"] == got["status"] == scfft.ERR_DIVERGED
    assert abs(got["iterations"] - ref["iterations"]) <= 2, (got["iterations"], ref["iterations"])
    if how == "overflow":
        assert not np.isfinite(got["residual"])


def test_non_finite_density_reports_divergence():
    rho = inputs.density_field(32, seed=5)
    rho[3, 7] = np.nan
    ref = osolver.solve(None, 20.0, [1, 0], "ms", tol=1e-10, max_iter=50,
                        sigma_field=1 + 19 * rho, sigma0=10.5)
    got = scfft.solve(density=rho, sigma1=20.0, e0=(1, 0), scheme="ms", sigma0=10.5, tol=1e-10,
                      max_iter=50)
    assert ref["status"] == got["status"] == scfft.ERR_DIVERGED
    assert ref["iterations"] == got["iterations"] == 1
