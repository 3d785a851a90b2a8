"""The solve loop: replayed graphs of 2^b iterations against direct launches.

A solve of max_iter = m runs m + 1 passes, replayed as the graphs of 2^b
iterations whose sizes add up to each check interval (the largest, at most
64, repeated).  Every combination of lengths and check intervals below must
stop at the same iterate with bit-identical sigma* and histories as the
same kernels launched one by one (SCFFT_NO_GRAPH), for a single solve and
for a batch (whose graph runs its problems as parallel branches).
"""
import numpy as np
import pytest

from paper_2001_08289_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2001_08289_amd import scfft  # noqa: E402


def _run(env, graph, **kw):
    if graph:
        env.delenv("SCFFT_NO_GRAPH", raising=False)
    else:
        env.setenv("SCFFT_NO_GRAPH", "1")
    return kw.pop("fn")(**kw)


@pytest.fixture
def env(monkeypatch):
    monkeypatch.delenv("SCFFT_NO_GRAPH", raising=False)
    scfft.release()
    yield monkeypatch
    scfft.release()


def test_fixed_lengths_and_check_intervals(env):
    chi = inputs.random_phase((64, 96), 0.3, seed=31)
    for check_every in (1, 7, 64, 100):
        for max_iter in (0, 1, 5, 19, 63, 64, 65, 130):
            out = []
            for graph in (True, False):
                r = _run(env, graph, fn=scfft.solve, phase=chi, sigma1=3 + 1j, e0=(1, 0),
                         scheme="acc_em", precision="fp64", tol=-1, max_iter=max_iter,
                         stag_window=0, div_factor=0, check_every=check_every, fields=False)
                out.append(r)
            a, b = out
            assert a["iterations"] == b["iterations"] == max_iter, (check_every, max_iter)
            assert a["sigma_star"] == b["sigma_star"], (check_every, max_iter)
            assert np.array_equal(a["residual_history"], b["residual_history"], equal_nan=True)


def test_converged_stop_matches_direct_launches(env):
    chi = inputs.square_array(128)
    for check_every in (1, 5, 16, 64):
        for precision, tol in (("fp64", 1e-10), ("fp32", 1e-6)):
            out = [_run(env, g, fn=scfft.solve, phase=chi, sigma1=100.0, e0=(1, 0),
                        scheme="acc_em", precision=precision, tol=tol, max_iter=500,
                        check_every=check_every, fields=False) for g in (True, False)]
            assert out[0]["iterations"] == out[1]["iterations"]
            assert out[0]["sigma_star"] == out[1]["sigma_star"]


def test_batch_branches_match_direct_launches(env):
    chis = [torch.as_tensor(inputs.random_phase((n, n), 0.3, seed=40 + n)).cuda()
            for n in (64, 96, 128, 80, 48)]
    sig = np.array([[2 + 1j, 0.3 - 0.5j, 10.0]] * len(chis))
    out = []
    for graph in (True, False):
        rs = _run(env, graph, fn=scfft.solve_batch, phases=chis, sigma1s=sig, scheme="acc_em",
                  precision="fp64", tol=1e-9, max_iter=300, check_every=6)
        out.append([(r["iterations"], r["sigma_star"]) for r in rs])
    assert out[0] == out[1]
