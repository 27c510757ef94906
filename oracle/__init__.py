"""Plain, slow, FP64 CPU oracle for the FFT-preconditioned interface GMRES of
Jiang, Lian & Wang, "A FFT-based GMRES for fast solving of Poisson equation in
concatenated geometry" (arXiv 2509.23180).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP path; the only common
dependency is the seeded input generator module `workloads`, which holds none
of the method's arithmetic.

What the oracle computes, and why that is the right reference
------------------------------------------------------------
The method of the paper (Section 2.3 block system, the Schur-complement
equations and Algorithm 1) is exact block elimination of one linear system
followed by a Krylov solve of the reduced system; its answer is therefore the
solution of the global composite 5-point system.  The oracle writes that
definition out directly:

* `composite`  assembles the global 5-point Helmholtz-Poisson matrix on the
  composite grid (Section 2.1, central-difference scheme and its block
  matrix form, with kappa on the diagonal as in the model equation of the
  Introduction) and solves it by banded Cholesky / banded LU (LAPACK) or, for
  very large grids, SuperLU.
* `rect`       the single-rectangle Dirichlet operator, the dense sine
  transform and the closed-form eigenvalues (Section 2.1), and per-mode
  tridiagonal solves written as dense/banded solves.
* `schur`      the Schur complement of the global matrix onto the coupled
  (centre) subdomain, formed from the global matrix partition (Section 2.3),
  plus plain Arnoldi (modified Gram-Schmidt), Givens rotations and a reference
  right-preconditioned GMRES(m) (Section 2.4).
* `layout`     the user-facing per-rectangle ordering of unknowns, written from
  the C header's definition, so that results can be compared node by node.

Every function is pinned by `-m "not gpu"` tests against closed forms,
hand-derived fixtures, invariants and library routines.
"""

from . import composite, layout, rect, schur  # noqa: F401
