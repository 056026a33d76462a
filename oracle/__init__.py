"""CPU oracle for the hierarchically preconditioned eigensolver (TEST INFRASTRUCTURE).

This package is a plain, slow, float64 CPU implementation of what the GPU
library computes.  It exists only to check the GPU path: the test suite, the
entry-point smoke check and the benchmark's CPU-baseline leg may import it;
nothing in the product path does.  It shares no code with the GPU library
(no common kernels, helpers or tables); both sides read the same seeded
inputs from the separate ``workloads`` package.

Modules and the passages of the paper they follow:
  philox   counter-based random numbers (Philox4x32-10, Salmon et al. 2011)
           used for the Lanczos start vectors (Alg. 3/4 draw random vectors).
  energy   energy elements and patch energies (Sec. 2.1).
  mmd      partition, local bases Phi, Householder complements U, localized
           Psi, level operators A^(k), M^(k) and the accuracy schedule
           (Sec. 2.2-2.3; Sec. 5 parameter choice).
  krylov   CG / flexible PCG (Sec. 4, operator OP), general Lanczos with the
           M inner product (Alg. 3), implicit restart (Alg. 2), extension
           (Alg. 4), refinement (Alg. 5) and the level driver (Alg. 6).
  backward first-order perturbation gradient of the leftmost eigenpairs with
           respect to the stored entries of A (eigenvalue outer products,
           eigenvector adjoints by a CG solve on the complement of the
           computed eigenvectors); the paper gives no derivative.
  dense    the plain definition of the result (dense symmetric eigensolve)
           and per-eigenpair error measures.
  backward gradient of eigenvalues / eigenvector functionals w.r.t. A.

Parity status: every function is pinned by a test in tests/test_oracle_*.py
except where its docstring says "parity unpinned".
"""
