"""Seeded synthetic inputs shared by the HIP path, the tests and the oracle.

This module holds only workload generators: voxel phase maps, a smooth
density field and seeded random draws.  It contains none of the solver's
arithmetic (no scheme scalars, no Gamma operator, no iteration), so both the
GPU path and the CPU oracle can take their inputs from here without sharing
any of the method.

Conventions (used throughout the project):
  * a grid has d = 2 or 3 axes; axis 0 (x) is the fastest-varying index, so a
    voxel (x, y[, z]) sits at flat index x + n0*(y + n1*z);
  * numpy arrays are shaped (n1, n0) in 2D and (n2, n1, n0) in 3D;
  * a phase map is uint8 with 1 in the inclusion phase (conductivity sigma1)
    and 0 in the matrix (conductivity sigma2 = 1), the indicator chi(x) of the
    paper's section on the original subspace collection;
  * a voxel is phase 1 when its centre ((j + 1/2)/N, ...) lies in the
    inclusion.
"""
from __future__ import annotations

import numpy as np


def square_array(n: int) -> np.ndarray:
    """Centred square of side n/2 in an n x n periodic cell (area fraction 1/4).

    The periodic array of squares at 25% volume fraction is the paper's model
    example (section "The numerical example of Moulinec and Suquet",
    eq. J47a).  Voxels [n/4, 3n/4)^2 are phase 1.
    """
    if n % 4:
        raise ValueError("square_array needs n divisible by 4")
    chi = np.zeros((n, n), dtype=np.uint8)
    chi[n // 4: 3 * n // 4, n // 4: 3 * n // 4] = 1
    return chi


def cube_array(n: int) -> np.ndarray:
    """Centred cube at (about) 25% volume fraction in an n^3 periodic cell.

    Side L = round(0.25**(1/3) * n) voxels at offset (n - L)//2 (n = 256 gives
    L = 161, offset 47, fraction 0.24875).  Cubic symmetry keeps sigma* a
    scalar (section "The original subspace collection", isotropy assumption).
    """
    side = int(round(0.25 ** (1.0 / 3.0) * n))
    off = (n - side) // 2
    chi = np.zeros((n, n, n), dtype=np.uint8)
    chi[off:off + side, off:off + side, off:off + side] = 1
    return chi


def laminate(n: int, d: int, fraction: float = 0.25, axis: int = 0,
             seed: int | None = None) -> np.ndarray:
    """Layered medium whose phase depends only on the coordinate along `axis`.

    With seed=None the first round(fraction*n) layers are phase 1; with a seed
    a random subset of that many layers is chosen.  Laminates have the exact
    arithmetic / harmonic mean effective conductivities used as closed-form
    checks.
    """
    k = int(round(fraction * n))
    prof = np.zeros(n, dtype=np.uint8)
    if seed is None:
        prof[:k] = 1
    else:
        rng = np.random.default_rng(seed)
        prof[rng.choice(n, size=k, replace=False)] = 1
    shape = (n,) * d
    # numpy axis of grid axis `axis` is d-1-axis
    view = [1] * d
    view[d - 1 - axis] = n
    return np.broadcast_to(prof.reshape(view), shape).astype(np.uint8).copy()


def random_phase(shape, fraction: float = 0.3, seed: int = 0) -> np.ndarray:
    """Independent Bernoulli(fraction) voxels: a rough two-phase map."""
    rng = np.random.default_rng(seed)
    return (rng.random(shape) < fraction).astype(np.uint8)


def random_disks(n: int, seed: int, target_fraction: float = 0.30,
                 rmin: float = 0.03, rmax: float = 0.08,
                 gap: float = 2.0 / 256.0, max_tries: int = 200000):
    """Periodic random sequential addition of non-overlapping disks.

    Radii ~ U[rmin, rmax] (cell units), centres uniform, accepted when every
    periodic centre distance is at least r_i + r_j + gap, until the continuum
    area fraction reaches `target_fraction`.  Returns (chi, disks) where disks
    is an (m, 3) array of (cx, cy, r).  The disk list depends only on the
    seed; `n` only sets the voxel sampling.
    """
    rng = np.random.default_rng(seed)
    disks: list[tuple[float, float, float]] = []
    area = 0.0
    tries = 0
    while area < target_fraction:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random_disks: could not reach the target fraction")
        cx, cy = rng.random(2)
        r = rmin + (rmax - rmin) * rng.random()
        ok = True
        for (px, py, pr) in disks:
            dx = abs(cx - px)
            dx = min(dx, 1.0 - dx)
            dy = abs(cy - py)
            dy = min(dy, 1.0 - dy)
            if dx * dx + dy * dy < (r + pr + gap) ** 2:
                ok = False
                break
        if ok:
            disks.append((cx, cy, r))
            area += np.pi * r * r
    d = np.array(disks, dtype=np.float64)
    xc = (np.arange(n) + 0.5) / n
    chi = np.zeros((n, n), dtype=np.uint8)
    for (cx, cy, r) in d:
        dx = np.abs(xc - cx)
        dx = np.minimum(dx, 1.0 - dx)
        dy = np.abs(xc - cy)
        dy = np.minimum(dy, 1.0 - dy)
        chi |= ((dy[:, None] ** 2 + dx[None, :] ** 2) <= r * r).astype(np.uint8)
    return chi, d


# Grid sizes (5-smooth) of the mixed-size batch of disk microstructures.
BATCH_GRIDS = (256, 288, 320, 360, 384, 400, 432, 480, 512, 576, 640, 720,
               768, 800, 900, 1024)


def density_field(n: int, seed: int = 5, length: float = 0.05,
                  mean: float = 0.5, amp: float = 0.3) -> np.ndarray:
    """Seeded smooth phase density rho(x) in [0, 1] on an n x n grid.

    White noise w ~ N(0,1) per voxel, filtered periodically with the Fourier
    multiplier exp(-2 pi^2 length^2 |m|^2) (a Gaussian of standard deviation
    `length` cells), standardised, then rho = clip(mean + amp*w, 0, 1).
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n))
    m = np.fft.fftfreq(n, d=1.0 / n)
    mult = np.exp(-2.0 * np.pi ** 2 * length ** 2 * (m[:, None] ** 2 + m[None, :] ** 2))
    wf = np.fft.ifft2(np.fft.fft2(w) * mult).real
    wf = (wf - wf.mean()) / wf.std()
    return np.clip(mean + amp * wf, 0.0, 1.0)


def smooth_direction(n: int, seed: int = 11, length: float = 0.05) -> np.ndarray:
    """Seeded smooth zero-mean unit-RMS field, a direction for finite differences."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n))
    m = np.fft.fftfreq(n, d=1.0 / n)
    mult = np.exp(-2.0 * np.pi ** 2 * length ** 2 * (m[:, None] ** 2 + m[None, :] ** 2))
    wf = np.fft.ifft2(np.fft.fft2(w) * mult).real
    return (wf - wf.mean()) / wf.std()


def contour_points(count: int, radius: float) -> np.ndarray:
    """Points z_j = radius * exp(2 pi i (j + 1/2)/count) on a circle in the z-plane."""
    j = np.arange(count)
    return radius * np.exp(2j * np.pi * (j + 0.5) / count)
