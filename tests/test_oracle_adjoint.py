"""Pins of oracle/adjoint.py.

* The adjoint solve equals a sparse direct solve with A^H.
* Complex symmetry of the ECS operator, W A = (W A)^T with W diagonal, gives
  A^{-H} g = conj(W) conj(A^{-1} (W^{-1} conj(g))): the adjoint solution must
  equal a transformed forward solve (independent of the conjugate-transposed
  hierarchy the oracle builds).
* The gradient Re(conj(lambda) u) of L = 0.5 ||P u - d||^2 matches central
  differences made exact for this rank-one change by Sherman-Morrison, and the
  Taylor remainder of L(k^2 + t v) decays as t^2.
"""

import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import adjoint as AD
from oracle import helmholtz as H
from oracle import krylov as K
from oracle import cycle as C
from paper_1211_4752_amd import workloads as W


def _setup(n=31, ecs=4, nshots=3):
    wl = W.heterogeneous_2d(n, nshots, ecs=ecs)
    prob = H.Problem(wl.n, wl.h, wl.k2, (ecs,) * 2, (ecs,) * 2, wl.ecs_angle)
    return prob, wl


def test_adjoint_solve_matches_direct():
    prob, wl = _setup()
    levels = H.build_hierarchy(prob)
    rng = np.random.default_rng(4)
    g = rng.standard_normal(levels[0].size) + 1j * rng.standard_normal(levels[0].size)
    lam, hist, its, status = AD.adjoint_solve(levels, g, rtol=1e-11)
    assert status == "converged"
    exact = spla.spsolve(levels[0].A.conj().T.tocsc(), g)
    assert np.linalg.norm(lam - exact) / np.linalg.norm(exact) < 1e-8


def test_adjoint_equals_transformed_forward_solve():
    prob, wl = _setup()
    levels = H.build_hierarchy(prob)
    lev = levels[0]
    Wd = np.multiply.outer(lev.weights[1], lev.weights[0]).ravel()
    rng = np.random.default_rng(5)
    g = rng.standard_normal(lev.size) + 1j * rng.standard_normal(lev.size)
    lam, *_ = AD.adjoint_solve(levels, g, rtol=1e-12)
    vc = C.VCycle(levels)
    y, *_ = K.gmres(lev.A, vc.precondition, np.conj(g) / Wd, rtol=1e-12, restart=20, maxit=5000)
    want = np.conj(Wd) * np.conj(y)
    assert np.linalg.norm(lam - want) / np.linalg.norm(want) < 1e-9


def _loss_and_grad(levels, prob, fs, P, ds):
    vc = C.VCycle(levels)
    A = levels[0].A
    us, lams = [], []
    for f, d in zip(fs, ds):
        u, *_ = K.gmres(A, vc.precondition, f, rtol=1e-12, restart=20, maxit=5000)
        us.append(u)
        lam, *_ = AD.adjoint_solve(levels, AD.receiver_grad_u(u, P, d), rtol=1e-12)
        lams.append(lam)
    return us, AD.receiver_loss(us, P, ds), AD.grad_k2(us, lams)


def _receivers(n, rows):
    import scipy.sparse as sp
    idx = [r * n + c for r, c in rows]
    return sp.csr_matrix((np.ones(len(idx)), (np.arange(len(idx)), idx)), shape=(len(idx), n * n))


def test_gradient_sherman_morrison_central_differences():
    prob, wl = _setup()
    n = prob.n[0]
    levels = H.build_hierarchy(prob)
    A = levels[0].A
    P = _receivers(n, [(25, c) for c in range(5, 26, 2)])
    fs = [f.ravel() for f in wl.f]
    rng = np.random.default_rng(6)
    ds = [P @ (rng.standard_normal(n * n) * 1e-3) for _ in fs]
    us, L0, g = _loss_and_grad(levels, prob, fs, P, ds)
    for i in rng.choice(np.arange(5 * n, n * n - 5 * n), 6, replace=False):
        eps = 1e-4 * prob.k2.ravel()[i]
        e = np.zeros(n * n, complex)
        e[i] = 1
        z = spla.spsolve(A.tocsc(), e)
        # A(k2 + t e_i) = A - t e_i e_i^T, so u(t) = u + t u_i / (1 - t z_i) z
        diff = 0.0
        for t in (eps, -eps):
            Lt = 0.0
            for u, d in zip(us, ds):
                delta = t * u[i] / (1 - t * z[i]) * z
                r = P @ u - d
                Pd = P @ delta
                Lt += float(np.real(np.vdot(r, Pd)) + 0.5 * np.linalg.norm(Pd) ** 2)
            diff += Lt if t > 0 else -Lt
        fd = diff / (2 * eps)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-12 * np.abs(g).max())


def test_gradient_taylor_remainder():
    prob, wl = _setup(nshots=2)
    n = prob.n[0]
    P = _receivers(n, [(20, c) for c in range(4, 27, 3)])
    fs = [f.ravel() for f in wl.f]
    rng = np.random.default_rng(7)
    ds = [P @ (rng.standard_normal(n * n) * 1e-3) for _ in fs]
    levels = H.build_hierarchy(prob)
    us, L0, g = _loss_and_grad(levels, prob, fs, P, ds)
    v = rng.standard_normal(n * n) * prob.k2.mean()
    rem = []
    for t in (1e-4, 5e-5, 2.5e-5):
        p2 = H.Problem(prob.n, prob.h, prob.k2 + t * v.reshape(prob.k2.shape), prob.ecs_lo,
                       prob.ecs_hi, prob.ecs_angle)
        A2 = H.operator(p2)
        ut = [spla.spsolve(A2.tocsc(), f) for f in fs]
        Lt = AD.receiver_loss(ut, P, ds)
        rem.append(abs(Lt - L0 - t * g @ v))
    assert rem[0] / rem[1] == pytest.approx(4.0, rel=0.1)
    assert rem[1] / rem[2] == pytest.approx(4.0, rel=0.1)
