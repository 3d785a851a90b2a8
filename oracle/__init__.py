"""CPU reference oracle for the FFT-based composite-conductivity solvers.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP library.

It is a plain, slow, fp64 numpy implementation of what the paper's method
computes, written step by step from the paper (G. W. Milton, "Substitution of
subspace collections with nonorthogonal subspaces to accelerate Fast Fourier
Transform methods applied to conducting composites"):

  fft       own mixed-radix FFT (decimation in time), direct DFT for primes
  scalars   the slit map t (eq. J3/J6/J23), p from (alpha, beta) (eq. J24),
            z-variables (eqs. J1, J2, J4), E2', J3' (eqs. J21, J26), closed
            forms (eq. J47a, laminates, Hashin-Shtrikman)
  symbols   discrete Gamma_1 symbol per Fourier mode (eq. J11 on a grid)
  solver    Moulinec-Suquet (eq. J0-0), Eyre-Milton (eq. J2), and both
            schemes run in the substituted space H'' (eqs. J27-J45)
  dense     brute-force dense solve of the discrete Lippmann-Schwinger system
  interval  power-iteration estimate of the singularity interval
  gradient  d sigma*/d sigma(x) and the adjoint solve

Every function that has no independent pin says "parity unpinned" in its
docstring.
"""
