"""Transfers, smoother and the level-dependent V(nu1, nu2) cycle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* Full-weighting restriction I_h^{2h} and (bi/tri)linear prolongation
  I_{2h}^h = 2^d (I_h^{2h})^T on vertex-centred grids, coarse point I sitting
  on fine point 2I+1 (Sec. 2.1, the transfer operators named after
  eq. standardtg).
* omega-Jacobi relaxation R_omega = I - omega D^{-1} A~ (Sec. 3.2.1,
  eq. wjacobi), D the diagonal of the level operator.
* GMRES(m) as the smoother (Sec. 3.2.1 and 3.2.2): one application is one
  GMRES cycle of m steps started from the current iterate, i.e. the iterate
  u + z, z in the Krylov space K_m(A~, r) with r = f - A~ u, of least
  residual norm; its residual is p_m(A~) r with a degree-m polynomial,
  p_m(0) = 1, whose coefficients are chosen anew on every application and on
  every level.  Arnoldi with modified Gram-Schmidt; the (m+1) x m
  least-squares problem is handed to a library solver.
* Two-grid correction with a perturbed coarse problem, applied recursively:
  on level l the operator is A~_l, the coarse problem is A~_{l+1} e = c R r
  with c = 1 for the CSL variant (Sec. 3.1, eq. cslvariant and eq. erreq1),
  and the correction is v <- v + P e (Sec. 3.1).  The coarsest level is
  solved directly.
* Standalone iteration of V-cycles started from u = 0 (Sec. 4.1): the
  residual ||f - A u|| / ||f|| of the incoming iterate is recorded as each
  cycle starts; the iteration stops after the first cycle whose incoming
  iterate met the tolerance (the returned iterate is that cycle's output, the
  reported count is the number of cycles before it), after the first cycle
  whose incoming ratio exceeded 1e8 or was not finite (diverged), or after
  maxit cycles.

Parity: pinned by tests/test_oracle_cycle.py (sine-mode transfer identities,
two-grid closed form with the corrected sign, smooth-mode factor, Poisson
invariant, brute-force error-propagation matrices, sparse direct solve).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


# ---------------------------------------------------------------------------
# Transfers (Sec. 2.1)
# ---------------------------------------------------------------------------

def restriction_1d(n_fine: int) -> sp.csr_matrix:
    """Full weighting (1/4, 1/2, 1/4): coarse I gathers fine 2I, 2I+1, 2I+2."""
    n_c = (n_fine - 1) // 2
    rows, cols, vals = [], [], []
    for I in range(n_c):
        for off, w in ((0, 0.25), (1, 0.5), (2, 0.25)):
            rows.append(I)
            cols.append(2 * I + off)
            vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n_c, n_fine))


def restriction(n_fine) -> sp.csr_matrix:
    """Tensor-product full weighting on a grid with x fastest."""
    R = None
    for a in reversed(range(len(n_fine))):     # slowest axis first
        r1 = restriction_1d(n_fine[a])
        R = r1 if R is None else sp.kron(R, r1, format="csr")
    return R.tocsr()


def prolongation(n_fine) -> sp.csr_matrix:
    """(Bi/tri)linear interpolation, P = 2^d R^T."""
    return (2.0 ** len(n_fine)) * restriction(n_fine).T.tocsr()


# ---------------------------------------------------------------------------
# Smoother (Sec. 3.2.1)
# ---------------------------------------------------------------------------

def jacobi(A, D, u, f, omega):
    """One omega-Jacobi sweep: u + omega D^{-1} (f - A u)  (eq. wjacobi)."""
    return u + omega * (f - A @ u) / D


def gmres_smooth(A, u, f, m=3):
    """One GMRES(m) smoothing step (Sec. 3.2.2): argmin over u + K_m(A, r) of
    ||f - A v||, r = f - A u.  Vectors stay in the dtype of u (complex64 in
    the mixed-precision inner cycle); the Hessenberg matrix and the small
    least-squares solve are complex128.  An exact breakdown (the Krylov space
    is invariant after j < m steps) ends the Arnoldi process early."""
    dt = u.dtype.type
    r = f - A @ u
    beta = float(np.linalg.norm(r))
    if beta == 0.0:
        return u
    V = [r / dt(beta)]
    H = np.zeros((m + 1, m), dtype=np.complex128)
    k = m
    for j in range(m):
        w = A @ V[j]
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], w)
            w = w - dt(H[i, j]) * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] == 0:
            k = j + 1
            break
        V.append(w / dt(H[j + 1, j]))
    rhs = np.zeros(k + 1, dtype=np.complex128)
    rhs[0] = beta
    y = np.linalg.lstsq(H[:k + 1, :k], rhs, rcond=None)[0]
    z = np.zeros_like(u)
    for i in range(k):
        z = z + dt(y[i]) * V[i]
    return u + z


# ---------------------------------------------------------------------------
# V-cycle (Sec. 3.1)
# ---------------------------------------------------------------------------

class VCycle:
    """Level-dependent V(nu1, nu2) cycle on a hierarchy from helmholtz.build_hierarchy.

    ``dtype`` selects the arithmetic of smoothing, transfers and the coarse
    levels (complex128, or complex64 for the mixed-precision inner cycle); the
    coarsest direct solve is always done in complex128 and rounded back.
    ``adjoint=True`` uses the conjugate-transposed level operators A~_l^H.
    ``smoother`` is "jacobi" (omega-Jacobi) or "gmres" (GMRES(degree)); with
    the latter the cycle is a nonlinear map of its right-hand side.
    """

    def __init__(self, levels, nu1=1, nu2=1, omega=2.0 / 3.0,
                 dtype=np.complex128, adjoint=False, rhs_scale=1.0, smoother="jacobi", degree=3):
        if smoother not in ("jacobi", "gmres"):
            raise ValueError(smoother)
        self.smoother, self.degree = smoother, degree
        self.levels = levels
        self.nu1, self.nu2 = nu1, nu2
        self.dtype = np.dtype(dtype)
        self.omega = self.dtype.type(omega)
        self.rhs_scale = rhs_scale   # c of eq. erreq1 (1 for CSL)
        self.A, self.D, self.R, self.P = [], [], [], []
        for l, lev in enumerate(levels):
            A = lev.A.conj().T.tocsr() if adjoint else lev.A
            self.A.append(A.astype(self.dtype))
            self.D.append(A.diagonal().astype(self.dtype))
            if l + 1 < len(levels):
                self.R.append(restriction(lev.n).astype(self.dtype))
                self.P.append(prolongation(lev.n).astype(self.dtype))
        Ac = levels[-1].A.conj().T if adjoint else levels[-1].A
        self.coarse = Ac.toarray().astype(np.complex128)

    def solve_coarsest(self, f):
        return np.linalg.solve(self.coarse, f.astype(np.complex128)).astype(self.dtype)

    def cycle(self, l, u, f):
        """One V(nu1, nu2) cycle on level l for A~_l u = f; returns the new u."""
        if l == len(self.levels) - 1:
            return self.solve_coarsest(f)
        A, D = self.A[l], self.D[l]
        for _ in range(self.nu1):
            u = self.smooth(A, D, u, f)
        r = f - A @ u
        fc = self.dtype.type(self.rhs_scale) * (self.R[l] @ r)
        e = self.cycle(l + 1, np.zeros_like(fc), fc)
        u = u + self.P[l] @ e
        for _ in range(self.nu2):
            u = self.smooth(A, D, u, f)
        return u

    def smooth(self, A, D, u, f):
        if self.smoother == "gmres":
            return gmres_smooth(A, u, f, self.degree)
        return jacobi(A, D, u, f, self.omega)

    def __call__(self, u, f):
        return self.cycle(0, u.astype(self.dtype), f.astype(self.dtype))

    def precondition(self, v):
        """M v: one cycle from a zero initial guess (Sec. 4.1, preconditioner use)."""
        return self.cycle(0, np.zeros(len(v), dtype=self.dtype), v.astype(self.dtype))


def residual_ratio(A, u, f) -> float:
    return float(np.linalg.norm(f - A @ u) / np.linalg.norm(f))


def standalone(vc: VCycle, f, u0=None, rtol=1e-6, maxit=100, div=1e8):
    """Standalone level-dependent multigrid iteration (Sec. 4.1).

    Returns (u, history, cycles, status) with status in
    {"converged", "not_converged", "diverged"}.  ``history[k]`` is the relative
    residual of the iterate entering cycle k; every recorded cycle has run, so
    a converged result is one cycle past the first iterate within rtol.
    """
    A0 = vc.A[0]
    u = np.zeros(len(f), dtype=vc.dtype) if u0 is None else u0.astype(vc.dtype)
    f = f.astype(vc.dtype)
    hist = []
    for k in range(maxit):
        rho = residual_ratio(A0, u, f)
        hist.append(rho)
        u = vc(u, f)
        if rho <= rtol:
            return u, np.array(hist), k, "converged"
        if not np.isfinite(rho) or rho > div:
            return u, np.array(hist), k, "diverged"
    return u, np.array(hist), maxit, "not_converged"
