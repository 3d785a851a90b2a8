"""The autotuner and the knobs it chooses among.

Every candidate the autotuner may pick -- x-pass register radix, Gamma-pass
radix and tile width, 3D y-pass tile width, packed column, padded pitch,
nontemporal streams -- is forced in turn (environment overrides, tuning
off) and must reproduce the oracle's iterates; the tuned plan itself is
checked against the oracle too, and its choice is reported and cached.
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

FORCE = ("SCFFT_XR", "SCFFT_GR", "SCFFT_LINE_C", "SCFFT_YC", "SCFFT_PACK", "SCFFT_PITCH",
         "SCFFT_NT", "SCFFT_TUNE", "SCFFT_R16")


def _err(got, ref):
    return np.abs(got["E"].cpu().numpy() - ref["E"]).max() / np.abs(ref["E"]).max()


@pytest.fixture
def clean_env(monkeypatch):
    for k in FORCE:
        monkeypatch.delenv(k, raising=False)
    scfft.release()
    yield monkeypatch
    scfft.release()


CASES = {
    "2d_real": ((64, 128), 10.0),
    "2d_complex": ((64, 128), 3 + 2j),
    "3d_real": ((16, 32, 64), 10.0),
}


@pytest.mark.parametrize("case", list(CASES))
def test_every_forced_candidate_matches_oracle(case, clean_env):
    shape, s1 = CASES[case]
    chi = inputs.random_phase(shape, 0.3, seed=12)
    e0 = (1, 0) if len(shape) == 2 else (1, 0, 0)
    ref = osolver.solve(chi, s1, list(e0), "acc_em", alpha=0.25, beta=4.0, tol=-1, max_iter=4,
                        stag_window=0, div_factor=0)
    clean_env.setenv("SCFFT_TUNE", "0")
    combos = []
    for xr in ("4", "8"):
        for gr in ("4", "8"):
            for c in ("1", "2", "4", "8"):
                combos.append({"SCFFT_XR": xr, "SCFFT_GR": gr, "SCFFT_LINE_C": c})
    if len(shape) == 3:
        combos += [{"SCFFT_YC": c, "SCFFT_LINE_C": "1"} for c in ("2", "4", "8")]
    combos += [{"SCFFT_PACK": "1"}, {"SCFFT_PITCH": "1"}, {"SCFFT_NT": "1"}]
    for env in combos:
        for k in FORCE[:-2]:
            clean_env.delenv(k, raising=False)
        for k, v in env.items():
            clean_env.setenv(k, v)
        scfft.release()
        for precision, bound in (("fp64", 1e-11), ("fp32", 2e-6)):
            got = scfft.solve(chi, s1, e0, "acc_em", precision=precision, tol=-1, max_iter=4,
                              stag_window=0, div_factor=0)
            assert _err(got, ref) < bound, (env, precision)
        info = scfft.plan_info(chi, s1, e0, "acc_em", precision="fp64")
        assert info["tuned"] == 0
        if "SCFFT_XR" in env:
            assert info["x_radix"] == int(env["SCFFT_XR"])
        if "SCFFT_GR" in env:
            assert info["gamma_radix"] == int(env["SCFFT_GR"])


def test_tuned_plans_match_oracle_and_are_reported(clean_env, tmp_path):
    cache = tmp_path / "tune.txt"
    clean_env.setenv("SCFFT_TUNE_CACHE", str(cache))
    # shapes no other test tunes, so each one is tuned (and cached) here
    for shape, s1, scheme in (((256, 512), 10.0, "acc_em"), ((90, 80), 10.0, "ms"),
                              ((32, 16, 64), 10.0, "acc_em"), ((80, 64), 2 + 1j, "em")):
        chi = inputs.random_phase(shape, 0.3, seed=13)
        e0 = (1, 0) if len(shape) == 2 else (1, 0, 0)
        for precision, bound in (("fp64", 1e-11), ("fp32", 2e-6)):
            info = scfft.plan_info(chi, s1, e0, scheme, precision=precision)
            assert info["tuned"] == 1, (shape, info)
            ref = osolver.solve(chi, s1, list(e0), scheme, alpha=0.25, beta=4.0, tol=-1,
                                max_iter=4, stag_window=0, div_factor=0)
            got = scfft.solve(chi, s1, e0, scheme, precision=precision, tol=-1, max_iter=4,
                              stag_window=0, div_factor=0)
            assert _err(got, ref) < bound, (shape, precision, info)
    lines = cache.read_text().splitlines()
    assert len(lines) >= 4 and all(len(ln.split()) == 17 for ln in lines)
    assert all(ln.startswith("gfx") for ln in lines)
