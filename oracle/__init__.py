"""CPU oracle for the level-dependent complex-shifted multigrid method.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
FP64 NumPy/SciPy statement of what the GPU path computes.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
it; the product library never calls it and shares no code with it.

Paper: S. Cools, B. Reps, W. Vanroose, "A new level-dependent coarse grid
correction scheme for indefinite Helmholtz problems", NLAA 2013
(arXiv:1211.4752).  Each function cites the section / equation it follows.

Modules
-------
helmholtz  discretisation: ECS node map, per-axis 3-point coefficients,
           shifted operators, hierarchy, shift schedule            (Sec. 2, 3.1)
cycle      full weighting, linear interpolation, omega-Jacobi,
           level-dependent V(nu1,nu2) cycle, standalone iteration (Sec. 2.1, 3.1, 3.2)
krylov     restarted right-preconditioned GMRES(m) with MGS      (Sec. 2.2, 4.1)
adjoint    conjugate-transposed hierarchy, adjoint solve and the
           pointwise gradient of a loss with respect to k^2       (extension)

Parity status of every function is listed in the module headers; all are
pinned by the `-m "not gpu"` tests in tests/test_oracle_*.py.
"""

from . import helmholtz, cycle, krylov, adjoint  # noqa: F401
