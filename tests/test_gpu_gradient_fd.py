"""Adjoint gradients of sigma* against finite differences of forward solves.

d sigma* / d rho(x) for sigma(x) = 1 + (sigma1 - 1) rho(x) (the adjoint
identity behind the derivative of the energy form of sigma*, eq. J13): the
single-precision adjoint gradient along a smooth direction against a
double-precision central difference, a single-precision central difference
against the double-precision gradient, and single voxels (inside each phase
and on the interface) of a 128^2 grid in double precision.
"""
import numpy as np
import pytest

from paper_2001_08289_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2001_08289_amd import scfft  # noqa: E402

S1 = 20.0
S0 = float(np.sqrt(S1))


def _sigma(rho, precision="fp64", tol=1e-13):
    return scfft.solve(density=rho, sigma1=S1, e0=(1, 0), scheme="em", sigma0=S0,
                       precision=precision, tol=tol, max_iter=4000, fields=False)["sigma_star"].real


def test_directional_derivative_fp32():
    n = 64
    rho = torch.tensor(inputs.density_field(n, seed=7), dtype=torch.float64, device="cuda")
    u = torch.tensor(inputs.smooth_direction(n, seed=13), dtype=torch.float64, device="cuda")
    g32 = scfft.gradient(density=rho, sigma1=S1, e0=(1, 0), precision="fp32", tol=1e-6,
                         max_iter=3000, sigma0=S0)["drho"].real
    g64 = scfft.gradient(density=rho, sigma1=S1, e0=(1, 0), precision="fp64", tol=1e-12,
                         max_iter=3000, sigma0=S0)["drho"].real
    eps = 1e-5
    fd64 = (_sigma(rho + eps * u) - _sigma(rho - eps * u)) / (2 * eps)
    an32 = (g32 * u).sum().item()
    an64 = (g64 * u).sum().item()
    assert abs(an64 - fd64) < 1e-7 * abs(fd64)
    # fp32 adjoint: fields stored in fp32 at a 1e-6 stopping increment
    assert abs(an32 - fd64) < 2e-5 * abs(fd64)
    # fp32 forward solves: the difference quotient carries their rounding
    # (about 1e-8 relative in sigma*) divided by the step, and a truncation
    # error of order h^2 (4 % at h = 2e-2, where rho + h u leaves [0, 1])
    h = 2e-3
    fd32 = (_sigma(rho + h * u, "fp32", 1e-7) - _sigma(rho - h * u, "fp32", 1e-7)) / (2 * h)
    assert abs(fd32 - an64) < 2e-3 * abs(an64)


def test_single_voxel_derivatives_fp64():
    n = 128
    rho_np = inputs.density_field(n, seed=9)
    rho = torch.tensor(rho_np, dtype=torch.float64, device="cuda")
    g = scfft.gradient(density=rho, sigma1=S1, e0=(1, 0), precision="fp64", tol=1e-13,
                       max_iter=4000, sigma0=S0)["drho"].real.cpu().numpy()
    # a voxel of each phase and the one where rho is closest to 1/2
    picks = [np.unravel_index(np.argmax(rho_np), rho_np.shape),
             np.unravel_index(np.argmin(rho_np), rho_np.shape),
             np.unravel_index(np.argmin(np.abs(rho_np - 0.5)), rho_np.shape)]
    def central(v, h):
        up, dn = rho.clone(), rho.clone()
        up[v] += h
        dn[v] -= h
        return (_sigma(up) - _sigma(dn)) / (2 * h)

    # one voxel's own polarisation makes sigma* markedly curved in its
    # density: the central difference keeps an O(h^2) error (about 6e-5
    # relative at h = 1e-3), which Richardson extrapolation over h and h/2
    # removes
    h = 1e-3
    for v in picks:
        d1, d2 = central(v, h), central(v, h / 2)
        rich = (4 * d2 - d1) / 3
        assert abs(d1 - g[v]) < 2e-4 * abs(g[v]), (v, d1, g[v])
        assert abs(rich - g[v]) < 2e-6 * abs(g[v]), (v, rich, g[v])
