"""Pins of the GMRES(m) smoother (oracle/cycle.py) and flexible GMRES
(oracle/krylov.py).

* One smoothing application is the least-squares minimiser of ||f - A v||
  over v in u + K_m(A, r) (Sec. 3.2.2): checked against a brute-force
  least-squares solve on the explicit power basis [r, A r, ..., A^{m-1} r]
  (an independent formulation), the closed form of m = 1 (minimal-residual
  step), exactness when A has at most m distinct eigenvalues (the residual
  polynomial can vanish on the whole spectrum), residual monotonicity and
  homogeneity.
* Sec. 3.2.2's argument against a fixed first-order smoother: where the
  spectrum of D^{-1} A~ straddles zero no real omega makes omega-Jacobi
  stable, while a GMRES(3) application never increases the residual.
* The V-cycle with the GMRES(3) smoother converges as a standalone solver on
  an ECS problem to the sparse direct solution.
* Flexible GMRES equals right-preconditioned GMRES for a fixed linear
  preconditioner (same Krylov space, same minimisation), and with the
  nonlinear GMRES(3) cycle converges to the direct solution.
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import cycle as C
from oracle import helmholtz as H
from oracle import krylov as K
from paper_1211_4752_amd import workloads as W


def _rnd(n, rng):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def _ecs_level(n=31, ecs=4):
    wl = W.heterogeneous_2d(n, 1, ecs=ecs)
    prob = H.Problem(wl.n, wl.h, wl.k2, (ecs,) * 2, (ecs,) * 2, wl.ecs_angle)
    return H.build_hierarchy(prob), wl


def _matrices():
    rng = np.random.default_rng(0)
    dense = sp.csr_matrix(rng.standard_normal((40, 40)) + 1j * rng.standard_normal((40, 40)) + 8 * np.eye(40))
    levels, _ = _ecs_level()
    return [dense, levels[0].A, levels[1].A, levels[2].A]


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_smoother_is_least_squares_minimiser(m):
    rng = np.random.default_rng(m)
    for A in _matrices():
        n = A.shape[0]
        u, f = _rnd(n, rng), _rnd(n, rng)
        v = C.gmres_smooth(A, u, f, m)
        r = f - A @ u
        B = [r]
        for _ in range(m - 1):
            B.append(A @ B[-1])
        B = np.stack(B, 1)
        c = np.linalg.lstsq(A @ B, r, rcond=None)[0]
        want = u + B @ c
        # least-squares perturbation bound: the power basis is ill-conditioned
        kappa = np.linalg.cond(A @ B)
        assert np.linalg.norm(v - want) <= 1e-14 * kappa * np.linalg.norm(want) + 1e-12
        rmin = np.linalg.norm(r - (A @ B) @ c)
        assert abs(np.linalg.norm(f - A @ v) - rmin) <= 1e-9 * rmin


def test_smoother_degree_one_closed_form():
    rng = np.random.default_rng(5)
    for A in _matrices():
        n = A.shape[0]
        u, f = _rnd(n, rng), _rnd(n, rng)
        r = f - A @ u
        Ar = A @ r
        alpha = np.vdot(Ar, r) / np.vdot(Ar, Ar)
        np.testing.assert_allclose(C.gmres_smooth(A, u, f, 1), u + alpha * r, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("distinct", [1, 2, 3])
def test_smoother_exact_on_small_spectrum(distinct):
    rng = np.random.default_rng(distinct)
    lam = np.array([2 + 1j, -3 + 0.5j, 7 - 2j])[:distinct]
    Q, _ = np.linalg.qr(rng.standard_normal((24, 24)) + 1j * rng.standard_normal((24, 24)))
    d = np.repeat(lam, 24 // distinct + 1)[:24]
    A = sp.csr_matrix(Q @ np.diag(d) @ Q.conj().T)
    u, f = _rnd(24, rng), _rnd(24, rng)
    v = C.gmres_smooth(A, u, f, 3)
    assert np.linalg.norm(f - A @ v) <= 1e-10 * np.linalg.norm(f - A @ u)
    np.testing.assert_allclose(v, np.linalg.solve(A.toarray(), f), rtol=1e-9, atol=1e-9)


def test_smoother_monotone_and_homogeneous():
    rng = np.random.default_rng(9)
    for A in _matrices():
        n = A.shape[0]
        u, f = _rnd(n, rng), _rnd(n, rng)
        v = C.gmres_smooth(A, u, f, 3)
        assert np.linalg.norm(f - A @ v) <= np.linalg.norm(f - A @ u)
        s = 0.3 - 2.0j
        np.testing.assert_allclose(C.gmres_smooth(A, s * u, s * f, 3), s * v, rtol=1e-11, atol=1e-11)
    assert np.array_equal(C.gmres_smooth(A, u, A @ u, 3), u)       # zero residual: unchanged


def test_smoother_keeps_complex64():
    levels, _ = _ecs_level()
    A = levels[0].A
    rng = np.random.default_rng(3)
    f = _rnd(A.shape[0], rng)
    v32 = C.gmres_smooth(A.astype(np.complex64), np.zeros(A.shape[0], np.complex64), f.astype(np.complex64), 3)
    v64 = C.gmres_smooth(A, np.zeros(A.shape[0], complex), f, 3)
    assert v32.dtype == np.complex64
    assert np.linalg.norm(v32 - v64) <= 1e-5 * np.linalg.norm(v64)


def test_first_order_smoother_unstable_gmres_is_not():
    """Sec. 3.2.2: on the finest level of the Dirichlet k = 40 problem (63^2)
    the eigenvalues mu of D^{-1} A~ lie on both sides of zero, so no real
    omega gives |1 - omega mu| < 1 for all of them (omega-Jacobi at
    omega = 2/3 amplifies the smooth modes), while one GMRES(3) application
    never increases the residual."""
    wl = W.dirichlet_constant_2d(63, 40.0)
    prob = H.Problem(wl.n, wl.h, wl.k2, (0, 0), (0, 0), wl.ecs_angle)
    A = H.build_hierarchy(prob)[0].A
    Ad = A.toarray()
    D = np.diag(Ad)
    mu = np.linalg.eigvals(Ad / D[:, None])
    assert mu.real.min() < 0 < mu.real.max()
    for omega in np.linspace(-2, 2, 81):
        assert np.abs(1 - omega * mu).max() >= 1.0
    assert np.abs(1 - (2.0 / 3.0) * mu).max() > 1.0
    rng = np.random.default_rng(1)
    for _ in range(5):
        u, f = _rnd(len(D), rng), _rnd(len(D), rng)
        v = C.gmres_smooth(A, u, f, 3)
        assert np.linalg.norm(f - A @ v) < np.linalg.norm(f - A @ u)


def test_standalone_with_gmres_smoother_converges():
    levels, wl = _ecs_level(63, 4)
    vc = C.VCycle(levels, smoother="gmres")
    f = wl.f[0].ravel()
    u, hist, it, st = C.standalone(vc, f, rtol=1e-8, maxit=200)
    assert st == "converged"
    exact = spla.spsolve(levels[0].A.tocsc(), f)
    assert np.linalg.norm(u - exact) <= 1e-6 * np.linalg.norm(exact)


def test_fgmres_equals_gmres_for_linear_preconditioner():
    levels, wl = _ecs_level(63, 4)
    vc = C.VCycle(levels)
    f = wl.f[0].ravel()
    x1, h1, i1, s1 = K.gmres(levels[0].A, vc.precondition, f, rtol=1e-8, restart=10, maxit=300)
    x2, h2, i2, s2 = K.gmres(levels[0].A, vc.precondition, f, rtol=1e-8, restart=10, maxit=300, flexible=True)
    assert s1 == s2 == "converged" and i1 == i2
    np.testing.assert_allclose(h2, h1, rtol=1e-8, atol=1e-13)
    assert np.linalg.norm(x2 - x1) <= 1e-8 * np.linalg.norm(x1)


def test_fgmres_with_gmres_smoothed_cycle():
    levels, wl = _ecs_level(63, 4)
    vc = C.VCycle(levels, smoother="gmres")
    f = wl.f[0].ravel()
    A = levels[0].A
    x, hist, it, st = K.gmres(A, vc.precondition, f, rtol=1e-10, restart=20, maxit=300, flexible=True)
    assert st == "converged"
    assert np.linalg.norm(f - A @ x) <= 1e-10 * np.linalg.norm(f) * (1 + 1e-6)
    assert np.all(np.diff(hist[1:min(len(hist), 21)]) <= 1e-15)     # monotone within the first restart
    exact = spla.spsolve(A.tocsc(), f)
    assert np.linalg.norm(x - exact) <= 1e-7 * np.linalg.norm(exact)
