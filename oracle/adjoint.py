"""Adjoint solve and the gradient of a loss with respect to k^2.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Not part of the paper: this is the differentiation extension built on top of
its method.  For the finest operator A = -Delta^h - k^2 (sigma_0 = 1, eq. HH)
and u = A^{-1} f, a real loss L(u) with complex gradient g = dL/d(conj u)
(PyTorch's convention, e.g. g = P^T (P u - d) for L = 0.5 ||P u - d||^2) has
    lambda = A^{-H} g,
    dL/d(k^2)_i = Re(conj(lambda_i) u_i),
    dL/d f      = lambda,
because dA/d(k^2)_i = -e_i e_i^T gives du = A^{-1} e_i u_i d(k^2)_i.

The adjoint system is solved with the same method applied to the
conjugate-transposed hierarchy {A~_l^H} (shifts conj(sigma_l)), i.e.
cycle.VCycle(adjoint=True) as the preconditioner of GMRES on A^H.

Parity: pinned by tests/test_oracle_adjoint.py (sparse direct solve of the
adjoint system, the complex-symmetry identity A^H = conj(W) conj(A) conj(W)^{-1},
Sherman-Morrison central differences, Taylor remainder decay).
"""

from __future__ import annotations

import numpy as np

from .cycle import VCycle
from .krylov import gmres


def adjoint_solve(levels, g, rtol=1e-10, restart=20, maxit=5000, **cyc):
    """lambda = A_0^{-H} g by GMRES(restart) preconditioned by the adjoint cycle."""
    vc = VCycle(levels, adjoint=True, **cyc)
    AH = levels[0].A.conj().T.tocsr()
    return gmres(AH, vc.precondition, g, rtol=rtol, restart=restart, maxit=maxit)


def grad_k2(u_list, lam_list) -> np.ndarray:
    """Sum over shots of Re(conj(lambda_s) u_s), pointwise."""
    out = np.zeros(len(u_list[0]))
    for u, lam in zip(u_list, lam_list):
        out += np.real(np.conj(lam) * u)
    return out


def receiver_loss(u_list, P, d_list) -> float:
    """L = 0.5 sum_s ||P u_s - d_s||^2 with a real sampling matrix P."""
    return 0.5 * sum(float(np.linalg.norm(P @ u - d) ** 2)
                     for u, d in zip(u_list, d_list))


def receiver_grad_u(u, P, d):
    """dL/d(conj u) = P^T (P u - d) for the receiver loss."""
    return P.T @ (P @ u - d)
