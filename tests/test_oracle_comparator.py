"""Pins of the fixed-shift comparator (Sec. 2.2: CSL preconditioner
-Delta - (1 + i beta) k^2 used on every level, as in the MG-FGMRES rows of
Table 3).

* Closed form: with the exact inverse of the shifted operator, the
  preconditioned Dirichlet operator has eigenvalues
  (lambda - k^2) / (lambda - (1 + i beta) k^2), all on the circle
  |z - 1/2| = 1/2 whatever beta and k.
* The multigrid approximation of that inverse (one V-cycle with the shift
  on every level) preconditions GMRES to the sparse direct solution of the
  unshifted problem.
"""

import numpy as np
import scipy.sparse.linalg as spla

from oracle import cycle as C
from oracle import helmholtz as H
from oracle import krylov as K
from paper_1211_4752_amd import workloads as W


def test_exact_csl_spectrum_on_circle():
    for n, k, beta in [(15, 30.0, 0.5), (31, 40.0, 1.0), (15, 12.0, -0.3)]:
        wl = W.dirichlet_constant_2d(n, k)
        prob = H.Problem(wl.n, wl.h, wl.k2, (0, 0), (0, 0), wl.ecs_angle)
        A = H.operator(prob).toarray()
        Ms = H.operator(prob, sigma=1 + 1j * beta).toarray()
        z = np.linalg.eigvals(A @ np.linalg.inv(Ms))
        assert np.abs(np.abs(z - 0.5) - 0.5).max() < 1e-10


def test_fixed_shift_cycle_preconditions_gmres():
    wl = W.heterogeneous_2d(63, 1, ecs=4)
    prob = H.Problem(wl.n, wl.h, wl.k2, (4, 4), (4, 4), wl.ecs_angle)
    L = H.auto_levels(prob.n)
    for smoother, flexible in (("jacobi", False), ("gmres", True)):
        levels = H.build_hierarchy(prob, sigma=np.full(L, 1 + 0.5j))
        vc = C.VCycle(levels, smoother=smoother)
        A = H.operator(prob)
        f = wl.f[0].ravel()
        x, hist, it, st = K.gmres(A, vc.precondition, f, rtol=1e-10, restart=20, maxit=2000, flexible=flexible)
        assert st == "converged"
        exact = spla.spsolve(A.tocsc(), f)
        assert np.linalg.norm(x - exact) <= 1e-7 * np.linalg.norm(exact)


def test_csg_variant_is_iterate_identical_to_csl():
    """Sec. 3.1 CSG variant: level operators e^{-i theta_l} (-Delta) - k^2 =
    e^{-i theta_l} A~_l (CSL) with the coarse right-hand side scaled by
    c = e^{-i dtheta}; the scalings cancel level by level, so one cycle (either
    smoother: omega-Jacobi sees D^{-1} A, GMRES(3) a scaled Krylov space)
    gives the CSL iterate."""
    import dataclasses
    import math
    wl = W.heterogeneous_2d(63, 1, ecs=4)
    prob = H.Problem(wl.n, wl.h, wl.k2, (4, 4), (4, 4), wl.ecs_angle)
    levels = H.build_hierarchy(prob)
    L = len(levels)
    dtheta = (math.pi / 6) / L
    csg = [dataclasses.replace(lev, A=(np.exp(-1j * l * dtheta) * lev.A).tocsr()) for l, lev in enumerate(levels)]
    rng = np.random.default_rng(4)
    u0 = rng.standard_normal(63 * 63) + 1j * rng.standard_normal(63 * 63)
    f = wl.f[0].ravel()
    for smoother in ("jacobi", "gmres"):
        a = C.VCycle(levels, smoother=smoother)(u0, f)
        b = C.VCycle(csg, smoother=smoother, rhs_scale=np.exp(-1j * dtheta))(u0, f)
        assert np.abs(a - b).max() <= 1e-11 * np.abs(a).max()
