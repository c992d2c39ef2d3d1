"""Pins of oracle/krylov.py.

* The restarted right-preconditioned GMRES converges to the sparse direct
  solution; its estimate |g_{j+1}| equals the true residual of the update it
  would produce (for a linear preconditioner) and never increases within a
  restart (textbook properties of GMRES).
* Without restarts GMRES is exact after at most n steps (Krylov exactness).
* The iterative-refinement form of the standalone cycle reproduces the
  standalone iteration of oracle/cycle.py for the linear FP64 cycle.
* Mixed precision: the complex64 cycle as preconditioner still reaches an
  FP64-level residual, and the solution error against the FP64 direct
  solve is within the bound cond * residual.
"""

import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import cycle as C
from oracle import helmholtz as H
from oracle import krylov as K
from paper_1211_4752_amd import workloads as W


def _problem(n=63, ecs=4, seed=2):
    wl = W.heterogeneous_2d(n, 2, ecs=ecs, field_seed=seed)
    prob = H.Problem(wl.n, wl.h, wl.k2, (ecs,) * 2, (ecs,) * 2, wl.ecs_angle)
    return prob, wl


def test_givens_zeroes_second_entry():
    rng = np.random.default_rng(0)
    for _ in range(20):
        a, b = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        c, s = K.givens(a, b)
        assert abs(-np.conj(s) * a + c * b) < 1e-14
        assert abs(c * c + abs(s) ** 2 - 1) < 1e-14


@pytest.mark.parametrize("ortho", ["mgs", "cgs2"])
def test_gmres_matches_direct_solve(ortho):
    prob, wl = _problem()
    levels = H.build_hierarchy(prob)
    vc = C.VCycle(levels)
    A = levels[0].A
    f = wl.f[0].ravel()
    x, hist, its, status = K.gmres(A, vc.precondition, f, rtol=1e-10, restart=20, maxit=3000, ortho=ortho)
    assert status == "converged"
    exact = spla.spsolve(A.tocsc(), f)
    assert np.linalg.norm(f - A @ x) / np.linalg.norm(f) <= 1e-10
    assert np.linalg.norm(x - exact) / np.linalg.norm(exact) < 1e-7


def test_gmres_orthogonalisation_variants_agree():
    """MGS and CGS2 run the same iteration: equal counts, histories equal to
    rounding (1e-8 relative above an absolute floor of 1e-11 ||f||)."""
    prob, wl = _problem(31, 2)
    levels = H.build_hierarchy(prob)
    vc = C.VCycle(levels)
    A = levels[0].A
    f = wl.f[0].ravel()
    x1, h1, i1, s1 = K.gmres(A, vc.precondition, f, rtol=1e-8, restart=20, maxit=500)
    x2, h2, i2, s2 = K.gmres(A, vc.precondition, f, rtol=1e-8, restart=20, maxit=500, ortho="cgs2")
    assert (i1, s1) == (i2, s2)
    assert np.all(np.abs(h1 - h2) <= 1e-8 * h1 + 1e-11)
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) < 1e-9


def test_gmres_estimate_is_true_residual_and_monotone():
    prob, wl = _problem(31, 2)
    levels = H.build_hierarchy(prob)
    vc = C.VCycle(levels)
    A = levels[0].A
    f = wl.f[1].ravel()
    for m in (1, 3, 7, 12):
        x, hist, its, status = K.gmres(A, vc.precondition, f, rtol=0.0, restart=m, maxit=m)
        true = np.linalg.norm(f - A @ x) / np.linalg.norm(f)
        assert hist[-1] == pytest.approx(true, rel=1e-8)
        assert np.all(np.diff(hist) <= 1e-14)


def test_gmres_krylov_exactness():
    n = 15
    prob = H.Problem((n,), (1 / 16,), np.full(n, 300.0), (3,), (3,))
    A = H.operator(prob)
    f = np.arange(1, n + 1, dtype=complex)
    x, hist, its, status = K.gmres(A, lambda v: v, f, rtol=1e-12, restart=40, maxit=40)
    assert status == "converged" and its <= n


def test_refinement_form_equals_standalone():
    prob = H.Problem((31, 31), (1 / 32, 1 / 32), np.full((31, 31), 40.0), (4, 4), (4, 4))
    levels = H.build_hierarchy(prob)
    vc = C.VCycle(levels)
    f = np.zeros(31 * 31, complex)
    f[480] = 1
    u1, h1, k1, s1 = C.standalone(vc, f, rtol=1e-8, maxit=40)
    u2, h2, k2, s2 = K.refine_standalone(levels[0].A, vc.precondition, f, rtol=1e-8, maxit=40)
    assert (k1, s1) == (k2, s2)
    np.testing.assert_allclose(h1, h2, rtol=1e-6, atol=1e-15)
    np.testing.assert_allclose(u1, u2, rtol=0, atol=1e-11 * np.abs(u1).max())


def test_mixed_precision_gmres_reaches_fp64_residual():
    prob, wl = _problem()
    levels = H.build_hierarchy(prob)
    A = levels[0].A
    f = wl.f[0].ravel()
    vc32 = C.VCycle(levels, dtype=np.complex64)
    M32 = lambda v: vc32.precondition(v).astype(np.complex128)
    x, hist, its, status = K.gmres(A, M32, f, rtol=1e-11, restart=20, maxit=4000)
    assert status == "converged"
    exact = spla.spsolve(A.tocsc(), f)
    err = np.linalg.norm(x - exact) / np.linalg.norm(exact)
    res = np.linalg.norm(f - A @ x) / np.linalg.norm(f)
    assert res <= 1e-11
    sv = np.linalg.svd(A.toarray(), compute_uv=False)
    assert err <= sv[0] / sv[-1] * res
    assert err < 1e-6
    # the complex64 preconditioner costs few extra iterations
    vc64 = C.VCycle(levels)
    _, h64, its64, _ = K.gmres(A, vc64.precondition, f, rtol=1e-11, restart=20, maxit=4000)
    assert its <= 1.2 * its64 + 20
