"""Compile-time mixed-radix passes (2/3/5-smooth lengths).

Every field value after a few fixed iterations against the oracle, on grids
whose axes are instantiated lengths (radix sequences with 8, 4, 2, 5 and 3
passes, several tiles and a ragged last tile of columns and rows), in both
precisions: 2D full-complex fields, and 3D fields whose y and z passes
(full-complex and real-field mode) take the compile-time strided passes;
and, at the batch grids' own sizes and on a larger 3D grid, the same
iterations against the runtime-planned passes (oracle-pinned elsewhere)
with the plan report showing which engine ran.
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

SMOOTH = 2   # plan_info engine code of the compile-time mixed-radix passes


def _rel(got, ref):
    return np.abs(got - ref).max() / np.abs(ref).max()


@pytest.fixture
def env(monkeypatch):
    for k in ("SCFFT_NO_SMOOTH", "SCFFT_NO_P2", "SCFFT_LINE_C", "SCFFT_TUNE"):
        monkeypatch.delenv(k, raising=False)
    scfft.release()
    yield monkeypatch
    scfft.release()


@pytest.mark.parametrize("shape", [(48, 80), (90, 96), (120, 160), (180, 90), (240, 192),
                                   (360, 288)])
@pytest.mark.parametrize("scheme,s1", [("acc_em", 3 + 2j), ("ms", 10.0), ("em", -5 + 1j),
                                       ("acc_ms", 100.0)])
def test_smooth_passes_match_oracle(shape, scheme, s1, env):
    chi = inputs.random_phase(shape, 0.3, seed=21)
    if scheme == "em" and shape != (90, 96):
        pytest.skip("one grid per scheme beyond the accelerated ones")
    ref = osolver.solve(chi, s1, [1.0, 0.0], scheme, alpha=0.25, beta=4.0, tol=-1, max_iter=3,
                        stag_window=0, div_factor=0)
    info = scfft.plan_info(chi, s1, (1, 0), scheme, precision="fp64")
    assert info["x_engine"] == SMOOTH and info["gamma_engine"] == SMOOTH, info
    for precision, bound in (("fp64", 1e-11), ("fp32", 2e-6)):
        got = scfft.solve(chi, s1, (1, 0), scheme, precision=precision, tol=-1, max_iter=3,
                          stag_window=0, div_factor=0)
        assert _rel(got["E"].cpu().numpy(), ref["E"]) < bound, (precision, shape)
        assert _rel(got["J"].cpu().numpy(), ref["J"]) < bound, (precision, shape)
        assert abs(got["sigma_star"] - ref["sigma_star"]) / abs(ref["sigma_star"]) < bound


@pytest.mark.parametrize("n", [288, 400, 576, 720, 900])
def test_smooth_matches_runtime_planned_passes(n, env):
    chi = inputs.random_phase((n, n), 0.25, seed=22)
    out = {}
    for flag in (None, "1"):
        if flag:
            env.setenv("SCFFT_NO_SMOOTH", flag)
        else:
            env.delenv("SCFFT_NO_SMOOTH", raising=False)
        scfft.release()
        info = scfft.plan_info(chi, 2 + 3j, (1, 0), "acc_em", precision="fp64")
        assert info["x_engine"] == (0 if flag else SMOOTH), info
        r = scfft.solve(chi, 2 + 3j, (1, 0), "acc_em", precision="fp64", tol=-1, max_iter=4,
                        stag_window=0, div_factor=0)
        out[flag] = r["E"].cpu().numpy()
    assert _rel(out[None], out["1"]) < 1e-12


def test_smooth_batch_of_mixed_grids(env):
    # one batch over two instantiated sizes and one power of two, each solve
    # against its own single solve
    chis = [inputs.random_phase((n, n), 0.3, seed=23 + n) for n in (96, 160, 128)]
    sig = np.array([[3 + 1j, 0.5 - 2j]] * 3)
    res = scfft.solve_batch([torch.as_tensor(c).cuda() for c in chis], sig, scheme="acc_em",
                            precision="fp64", tol=1e-10, max_iter=400)
    for i, c in enumerate(chis):
        for j in range(2):
            one = scfft.solve(c, sig[i, j], (1, 0), "acc_em", precision="fp64", tol=1e-10,
                              max_iter=400, fields=False)
            got = res[i * 2 + j]["sigma_star"]
            assert abs(got - one["sigma_star"]) / abs(one["sigma_star"]) < 1e-12


@pytest.mark.parametrize("shape", [(12, 10, 48), (6, 8, 90)])
@pytest.mark.parametrize("scheme,s1", [("acc_em", 3 + 2j), ("ms", 10.0)])
def test_smooth_x_pass_in_3d(shape, scheme, s1, env):
    # 3D full-complex fields: the x pass takes the compile-time passes, the
    # strided y and z passes (10 and 12 points) the runtime-planned ones
    chi = inputs.random_phase(shape, 0.3, seed=24)
    ref = osolver.solve(chi, s1, [1.0, 0.0, 0.0], scheme, alpha=0.25, beta=4.0, tol=-1,
                        max_iter=3, stag_window=0, div_factor=0)
    info = scfft.plan_info(chi, s1, (1, 0, 0), scheme, precision="fp64")
    assert info["x_engine"] == SMOOTH and info["gamma_engine"] == 0, info
    assert info["y_engine"] == 0, info
    for precision, bound in (("fp64", 1e-11), ("fp32", 2e-6)):
        got = scfft.solve(chi, s1, (1, 0, 0), scheme, precision=precision, tol=-1, max_iter=3,
                          stag_window=0, div_factor=0)
        assert _rel(got["E"].cpu().numpy(), ref["E"]) < bound, (precision, shape)
        assert abs(got["sigma_star"] - ref["sigma_star"]) / abs(ref["sigma_star"]) < bound


@pytest.mark.parametrize("shape,scheme,s1,engines", [
    # full complex: x, y and z all instantiated lengths
    ((48, 90, 80), "acc_em", 3 + 2j, (SMOOTH, SMOOTH, SMOOTH)),
    ((48, 90, 80), "acc_ms", 0.2 + 1j, (SMOOTH, SMOOTH, SMOOTH)),
    ((48, 90, 80), "ms", 10.0, (SMOOTH, SMOOTH, SMOOTH)),
    # 30 columns: ragged last tiles in the y and z passes; runtime x pass
    ((96, 80, 30), "acc_em", 3 + 2j, (0, SMOOTH, SMOOTH)),
    # real-field mode: 33 half-spectrum columns, register x pass
    ((90, 48, 64), "ms", 10.0, (1, SMOOTH, SMOOTH)),
    ((90, 48, 64), "em", 0.05, (1, SMOOTH, SMOOTH)),
])
def test_smooth_strided_passes_in_3d(shape, scheme, s1, engines, env):
    # 3D Gamma pass (three components per mode) and forward / inverse y
    # passes through the compile-time passes, every field value against the
    # oracle after three fixed iterations
    chi = inputs.random_phase(shape, 0.3, seed=25)
    ref = osolver.solve(chi, s1, [1.0, 0.0, 0.0], scheme, alpha=0.25, beta=4.0, tol=-1,
                        max_iter=3, stag_window=0, div_factor=0)
    for precision, bound in (("fp64", 1e-11), ("fp32", 2e-6)):
        info = scfft.plan_info(chi, s1, (1, 0, 0), scheme, precision=precision)
        assert (info["x_engine"], info["y_engine"], info["gamma_engine"]) == engines, info
        got = scfft.solve(chi, s1, (1, 0, 0), scheme, precision=precision, tol=-1, max_iter=3,
                          stag_window=0, div_factor=0)
        assert _rel(got["E"].cpu().numpy(), ref["E"]) < bound, (precision, shape)
        assert _rel(got["J"].cpu().numpy(), ref["J"]) < bound, (precision, shape)
        assert abs(got["sigma_star"] - ref["sigma_star"]) / abs(ref["sigma_star"]) < bound


def test_smooth_3d_against_runtime_passes(env):
    # a larger 3D grid (many tiles per pass, both precisions): the same
    # iterations through the runtime-planned passes
    chi = inputs.random_phase((160, 192, 96), 0.3, seed=26)
    for precision, bound in (("fp64", 1e-12), ("fp32", 2e-6)):
        out = []
        for flag in (False, True):
            if flag:
                env.setenv("SCFFT_NO_SMOOTH", "1")
            else:
                env.delenv("SCFFT_NO_SMOOTH", raising=False)
            scfft.release()
            info = scfft.plan_info(chi, 2 + 3j, (1, 0, 0), "acc_em", precision=precision)
            assert info["y_engine"] == (0 if flag else SMOOTH), info
            assert info["gamma_engine"] == (0 if flag else SMOOTH), info
            out.append(scfft.solve(chi, 2 + 3j, (1, 0, 0), "acc_em", precision=precision, tol=-1,
                                   max_iter=6, stag_window=0, div_factor=0))
        a, b = out
        assert _rel(a["E"].cpu().numpy(), b["E"].cpu().numpy()) < bound, precision
        assert abs(a["sigma_star"] - b["sigma_star"]) / abs(b["sigma_star"]) < bound


def test_smooth_batch_of_3d_grids(env):
    # one batch over a 3D grid of instantiated lengths on every axis, one
    # with short 16-lane lines and a ragged tile, and a power-of-two grid,
    # each solve against its own single solve
    shapes = [(48, 90, 80), (96, 48, 30), (32, 32, 32)]
    chis = [inputs.random_phase(s, 0.3, seed=27 + i) for i, s in enumerate(shapes)]
    sig = np.array([[3 + 1j, 0.5 - 2j]] * 3)
    for precision, tol, bound in (("fp64", 1e-10, 1e-12), ("fp32", 1e-5, 1e-6)):
        res = scfft.solve_batch([torch.as_tensor(c).cuda() for c in chis], sig, e0=(1, 0, 0),
                                scheme="acc_em", precision=precision, tol=tol, max_iter=400)
        for i, c in enumerate(chis):
            for j in range(2):
                one = scfft.solve(c, sig[i, j], (1, 0, 0), "acc_em", precision=precision, tol=tol,
                                  max_iter=400, fields=False)
                got = res[i * 2 + j]
                assert got["iterations"] == one["iterations"], (precision, i, j)
                rel = abs(got["sigma_star"] - one["sigma_star"]) / abs(one["sigma_star"])
                assert rel < bound, (precision, i, j, rel)


@pytest.mark.parametrize("shape", [(90, 96), (180, 240), (64, 400), (48, 90, 80), (12, 10, 48)])
@pytest.mark.parametrize("scheme,s1", [("acc_em", 100.0), ("acc_ms", 0.05), ("ms", 10.0),
                                       ("em", 1000.0)])
def test_smooth_real_field_x_pass(shape, scheme, s1, env):
    # real sigma1 on a mixed-radix x length: real-field mode (two real rows
    # per complex line, half spectra in X) in 3D and for 2D fp64 (2D fp32
    # keeps full-complex fields), every field value against the oracle after
    # three fixed iterations
    chi = inputs.random_phase(shape, 0.3, seed=28)
    e0 = (1, 0) if len(shape) == 2 else (1, 0, 0)
    ref = osolver.solve(chi, s1, list(map(float, e0)), scheme, alpha=0.25, beta=4.0, tol=-1,
                        max_iter=3, stag_window=0, div_factor=0)
    for precision, bound in (("fp64", 1e-11), ("fp32", 2e-6)):
        info = scfft.plan_info(chi, s1, e0, scheme, precision=precision)
        real = 1 if (len(shape) == 3 or precision == "fp64") else 0
        assert info["real"] == real and info["x_engine"] == SMOOTH, info
        got = scfft.solve(chi, s1, e0, scheme, precision=precision, tol=-1, max_iter=3,
                          stag_window=0, div_factor=0)
        assert _rel(got["E"].cpu().numpy(), ref["E"]) < bound, (precision, shape)
        assert _rel(got["J"].cpu().numpy(), ref["J"]) < bound, (precision, shape)
        assert abs(got["sigma_star"] - ref["sigma_star"]) / abs(ref["sigma_star"]) < bound


def test_smooth_real_field_converged(env):
    # converged real-field solves on a mixed-radix grid against the
    # full-complex path (SCFFT_NO_REAL) and the oracle's sigma*
    chi = inputs.random_phase((160, 240), 0.3, seed=29)
    ref = osolver.solve(chi, 20.0, [1.0, 0.0], "acc_em", alpha=0.25, beta=4.0, tol=1e-12,
                        max_iter=300)
    out = []
    for flag in (False, True):
        if flag:
            env.setenv("SCFFT_NO_REAL", "1")
        scfft.release()
        assert scfft.plan_info(chi, 20.0, (1, 0), "acc_em", precision="fp64")["real"] == \
            (0 if flag else 1)
        out.append(scfft.solve(chi, 20.0, (1, 0), "acc_em", precision="fp64", tol=1e-11,
                               max_iter=300, fields=False))
    a, b = out
    assert a["status"] == 0 and a["iterations"] == b["iterations"]
    assert abs(a["sigma_star"] - b["sigma_star"]) < 1e-12 * abs(b["sigma_star"])
    assert abs(a["sigma_star"] - ref["sigma_star"]) < 1e-9 * abs(ref["sigma_star"])


def test_smooth_real_field_entry_points(env):
    # every entry point that iterates the x pass, in real-field mode on a
    # mixed-radix grid (96^2 fp64) against the same call on full-complex
    # fields (SCFFT_NO_REAL)
    chi = inputs.random_phase((96, 96), 0.3, seed=30)
    rho = torch.tensor(inputs.density_field(96, seed=31), dtype=torch.float64, device="cuda")
    out = []
    for flag in (False, True):
        if flag:
            env.setenv("SCFFT_NO_REAL", "1")
        else:
            env.delenv("SCFFT_NO_REAL", raising=False)
        scfft.release()
        assert scfft.plan_info(chi, 20.0, (1, 0), "em", precision="fp64")["real"] == \
            (0 if flag else 1)
        r = {}
        g = scfft.gradient(density=rho, sigma1=20.0, e0=(1, 0), precision="fp64", tol=1e-12,
                           max_iter=3000)
        r["drho"] = g["drho"].real.cpu().numpy()
        r["dsigma1"] = complex(g["dsigma1"])
        r["interval"] = scfft.estimate_interval(chi, iters=40)
        r["lanczos"] = scfft.lanczos(chi, (1, 0), steps=12)
        r["series"] = scfft.series_coefficients(chi, (1, 0), nterms=10)
        r["tensor"] = np.array(scfft.effective_tensor(chi, 20.0, "acc_em", tol=1e-12)["tensor"])
        out.append(r)
    a, b = out
    assert _rel(a["drho"], b["drho"]) < 1e-9
    assert abs(a["dsigma1"] - b["dsigma1"]) < 1e-10 * abs(b["dsigma1"])
    for k in ("alpha", "beta"):
        assert abs(a["interval"][k] - b["interval"][k]) < 1e-10 * abs(b["interval"][k])
    assert np.allclose(a["lanczos"]["a"], b["lanczos"]["a"], rtol=1e-10, atol=1e-12)
    assert np.allclose(a["lanczos"]["b"], b["lanczos"]["b"], rtol=1e-10, atol=1e-12)
    assert np.allclose(a["series"], b["series"], rtol=1e-10, atol=1e-12)
    assert np.allclose(a["tensor"], b["tensor"], rtol=1e-10, atol=1e-12)
