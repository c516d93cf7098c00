"""CPU oracle for the Helmholtz / encoder-solver hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 restatement of
what the paper's method computes, written to check the GPU library against.
Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import it; the product path never does, and it imports nothing from the
product package.

Modules
  operator   eq. (3.1)-(3.2): the 5-point Helmholtz matrix, its matrix-free
             stencil, a brute-force dense builder, the direct solve.
  multigrid  eq. (3.12) and Sec. 3.4: the shifted-Laplacian V-cycle (3 levels).
  krylov     GMRES / right-preconditioned flexible GMRES (restarted).
  unet       eq. (3.13), (3.14), (4.1) and Fig. 1: encoder and solver U-Nets,
             forward and backward in FP64.
  train      eq. (4.2)-(4.3), Alg. 2: MSE loss, Adam, data generation,
             light-weight retraining.
  fwi        eq. (3.5), (3.10) (corrected), (4.4)-(4.8): misfit and gradient.
  philox     Philox-4x32-10 counter-based generator (random draws of the method).

Functions whose result no independent pin fixes say "parity unpinned" in their
docstring.
"""
