"""Solves on a caller's stream (torch's current stream, passed through the
C ABI as opt->stream): the same bits as on the default stream, for a single
solve with fields and histories, a batch, and the no-allocation entry point,
with the graphs captured on that stream.
"""
import numpy as np
import pytest

from paper_2001_08289_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2001_08289_amd import scfft  # noqa: E402


def _solve(chi, **kw):
    return scfft.solve(chi, 3 + 1j, (1, 0), "acc_em", precision="fp64", tol=1e-10, max_iter=300,
                       check_every=8, **kw)


def test_single_solve_and_batch_on_a_user_stream():
    scfft.release()
    chi = torch.as_tensor(inputs.random_phase((96, 128), 0.3, seed=51)).cuda()
    chis = [torch.as_tensor(inputs.random_phase((n, n), 0.3, seed=52 + n)).cuda()
            for n in (64, 80, 128)]
    sig = np.array([[2 + 1j, 0.5 - 0.2j]] * 3)
    torch.cuda.synchronize()
    ref = _solve(chi)
    ref_b = scfft.solve_batch(chis, sig, scheme="acc_em", precision="fp64", tol=1e-9,
                              max_iter=300, check_every=6)
    ref_n = _solve(chi, noalloc=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        got = _solve(chi)
        got_b = scfft.solve_batch(chis, sig, scheme="acc_em", precision="fp64", tol=1e-9,
                                  max_iter=300, check_every=6)
        got_n = _solve(chi, noalloc=True)
    s.synchronize()
    for a, b in ((ref, got), (ref_n, got_n)):
        assert a["iterations"] == b["iterations"]
        assert a["sigma_star"] == b["sigma_star"]
        assert torch.equal(a["E"], b["E"]) and torch.equal(a["J"], b["J"])
        assert np.array_equal(a["residual_history"], b["residual_history"], equal_nan=True)
    assert [(r["iterations"], r["sigma_star"]) for r in ref_b] == \
        [(r["iterations"], r["sigma_star"]) for r in got_b]
    # the no-allocation path runs the same kernels without graphs
    assert abs(ref_n["sigma_star"] - ref["sigma_star"]) <= 1e-13 * abs(ref["sigma_star"])
    scfft.release()
