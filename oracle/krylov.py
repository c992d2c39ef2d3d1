"""Restarted right-preconditioned GMRES(m) and mixed-precision refinement.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper uses the level-dependent cycle both as a solver and as the
preconditioner of an outer Krylov method, one V(1,1) cycle per outer step
(Sec. 2.2 last paragraph, Sec. 3.2.2 last paragraph, Sec. 4.1 discussion of
Table 3).  With the fixed omega-Jacobi smoother the cycle is a fixed linear
map M, so right-preconditioned GMRES(m) is exact: x = x0 + M (V y).

This is the textbook algorithm (Saad & Schultz restarted GMRES) with modified
Gram-Schmidt and complex Givens rotations, written out step by step:

  r0 = f - A x0, beta = ||r0||, v_0 = r0 / beta, g = beta e_0
  for j = 0 .. m-1:
      w = A M v_j
      for i = 0 .. j:  H[i,j] = <v_i, w>,  w -= H[i,j] v_i
      H[j+1,j] = ||w||,  v_{j+1} = w / H[j+1,j]
      rotate column j by the previous rotations, build rotation j,
      g[j+1] = -conj(s_j) g[j],  g[j] = c_j g[j]
      residual estimate |g[j+1]| / ||f||
  y = H[:j+1,:j+1]^{-1} g[:j+1],  x += M (V y)

``ortho="cgs2"`` replaces the modified Gram-Schmidt loop by classical
Gram-Schmidt applied twice (h1 = V^H w, w -= V h1, h2 = V^H w, w -= V h2,
H[:, j] = h1 + h2); both are standard stable Arnoldi variants and serve to
measure how far two correct FP64 evaluations of the same iteration drift
apart.

``flexible=True`` is flexible GMRES (Saad 1993): z_j = M v_j is stored and
the update is x += Z y, which stays exact when M changes from step to step,
as the cycle with the GMRES(m) smoother does (Sec. 3.2.2 last paragraph).
For a fixed linear M it produces the same iterates as the right-
preconditioned form.

The history records ||f - A x0|| / ||f|| first, then the estimate after every
outer step (one preconditioner application each).  When the estimate meets
rtol the solution is updated and the true residual is checked; if it still
exceeds rtol the method restarts.

The mixed-precision mode evaluates M in complex64 (the cycle of
cycle.VCycle with dtype=complex64) while everything else stays complex128.

Parity: pinned by tests/test_oracle_krylov.py (sparse direct solve,
monotone residual within a restart, Krylov exactness on a small system).
"""

from __future__ import annotations

import numpy as np


def givens(a: complex, b: complex):
    """Complex rotation [[c, s], [-conj(s), c]] with c real zeroing b below a."""
    if b == 0:
        return 1.0, 0.0 + 0.0j
    if a == 0:
        return 0.0, np.conj(b) / abs(b)
    t = np.hypot(abs(a), abs(b))
    c = abs(a) / t
    s = (a / abs(a)) * np.conj(b) / t
    return c, s


def gmres(A, M, f, x0=None, rtol=1e-6, restart=20, maxit=1000, ortho="mgs", flexible=False):
    """Right-preconditioned restarted GMRES(restart) (FGMRES with flexible).

    ``A`` is a sparse matrix, ``M`` a callable v -> M v returning complex128,
    ``ortho`` "mgs" or "cgs2".  Returns (x, history, iterations, status).
    """
    if ortho not in ("mgs", "cgs2"):
        raise ValueError(ortho)
    f = np.asarray(f, dtype=np.complex128)
    nf = np.linalg.norm(f)
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.complex128)
    hist = []
    it = 0
    while True:
        r = f - A @ x
        beta = np.linalg.norm(r)
        if not hist:
            hist.append(beta / nf)
        if beta / nf <= rtol:
            return x, np.array(hist), it, "converged"
        if it >= maxit:
            return x, np.array(hist), it, "not_converged"
        m = restart
        V = np.zeros((m + 1, len(f)), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        Z = np.zeros((m, len(f)), dtype=np.complex128) if flexible else None
        j_end = 0
        for j in range(m):
            z = M(V[j])
            if flexible:
                Z[j] = z
            w = A @ z
            if ortho == "mgs":
                for i in range(j + 1):
                    H[i, j] = np.vdot(V[i], w)
                    w = w - H[i, j] * V[i]
            else:
                for _ in range(2):
                    h = V[:j + 1].conj() @ w
                    w = w - V[:j + 1].T @ h
                    H[:j + 1, j] += h
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                a, b = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * b
                H[i + 1, j] = -np.conj(sn[i]) * a + cs[i] * b
            cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            est = abs(g[j + 1]) / nf
            hist.append(est)
            j_end = j + 1
            if not np.isfinite(est):
                return x, np.array(hist), it, "diverged"
            if est <= rtol or it >= maxit:
                break
        k = j_end
        y = np.zeros(k, dtype=np.complex128)
        for i in reversed(range(k)):                # back substitution
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + (Z[:k].T @ y if flexible else M(V[:k].T @ y))


def refine_standalone(A, M, f, rtol=1e-6, maxit=100, div=1e8):
    """u_{k+1} = u_k + M (f - A u_k) with the residual and update in FP64.

    This is the standalone cycle written as iterative refinement: for a linear
    cycle it produces the same iterates as cycle.standalone; with M in
    complex64 it is the mixed-precision standalone solver.  Same stopping
    rules and history convention as cycle.standalone.
    """
    f = np.asarray(f, dtype=np.complex128)
    nf = np.linalg.norm(f)
    u = np.zeros_like(f)
    hist = []
    for k in range(maxit):
        r = f - A @ u
        rho = np.linalg.norm(r) / nf
        hist.append(rho)
        u = u + M(r).astype(np.complex128)
        if rho <= rtol:
            return u, np.array(hist), k, "converged"
        if not np.isfinite(rho) or rho > div:
            return u, np.array(hist), k, "diverged"
    return u, np.array(hist), maxit, "not_converged"
