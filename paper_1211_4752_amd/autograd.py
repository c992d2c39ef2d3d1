"""Differentiable Helmholtz solve: u = A(k^2)^{-1} f through the HIP library.

Forward: mg_solve (level-dependent multigrid preconditioned GMRES, or the
standalone cycle).  Backward: with g = dL/d(conj u) as PyTorch passes it for a
real loss (for L = 0.5 ||P u - d||^2, g = P^T (P u - d)),
    lambda = A^{-H} g                    (mg_solve_adjoint: the same cycle on the
                                          conjugate-transposed hierarchy)
    dL/d(k^2) = sum_rhs Re(conj(lambda) u)   (mg_grad_k2)
    dL/d f    = lambda
since A = -Delta^h - k^2 on the finest level (sigma_0 = 1) gives
dA/d(k^2)_i = -e_i e_i^T and du = A^{-1} e_i u_i d(k^2)_i.  This is an
extension of the paper's method (differentiation of the discrete solution).
"""

from __future__ import annotations

import math

import torch

from . import mg


class HelmholtzSolve(torch.autograd.Function):
    """u = HelmholtzSolve.apply(k2, f, opts) with opts a dict:

    n, h, ecs, ecs_angle, theta_max, omega, smoother ("gmres3" | "jacobi",
    default "gmres3", the paper's smoother), precision ("c128" | "mixed"),
    mode ("gmres" | "standalone"), rtol, maxit, restart, adjoint_rtol
    (defaults to rtol).
    k2: float64 device tensor shaped like the grid; f: complex128 device
    tensor (nrhs, *grid).  A solve that does not reach rtol raises.
    """

    @staticmethod
    def forward(ctx, k2, f, opts):
        k2 = k2.detach().contiguous()
        f = f.detach().contiguous()
        s = mg.Solver(opts["n"], opts["h"], k2, ecs=opts.get("ecs", 0),
                      ecs_angle=opts.get("ecs_angle", math.pi / 4),
                      theta_max=opts.get("theta_max", math.pi / 6), omega=opts.get("omega", 2.0 / 3.0),
                      nrhs=f.shape[0], smoother=opts.get("smoother", "gmres3"),
                      precision=opts.get("precision", "c128"))
        u = s.empty()
        st, its, _ = s.solve(u, f, mode=opts.get("mode", "gmres"), rtol=opts.get("rtol", 1e-10),
                             maxit=opts.get("maxit", 20000), restart=opts.get("restart", 20))
        if st != "converged":
            s.close()
            raise RuntimeError("forward Helmholtz solve %s after %s steps" % (st, its))
        ctx.solver = s
        ctx.opts = opts
        ctx.iters = its
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        s = ctx.solver
        opts = ctx.opts
        (u,) = ctx.saved_tensors
        lam = s.empty()
        st, its, _ = s.solve_adjoint(lam, grad_u.contiguous(), mode=opts.get("mode", "gmres"),
                                     rtol=opts.get("adjoint_rtol", opts.get("rtol", 1e-10)),
                                     maxit=opts.get("maxit", 20000), restart=opts.get("restart", 20))
        if st != "converged":
            raise RuntimeError("adjoint Helmholtz solve %s after %s steps" % (st, its))
        grad_k2 = torch.zeros_like(s.k2)
        s.grad_k2(u, lam, grad_k2)
        s.close()
        ctx.solver = None
        return grad_k2, lam, None


def helmholtz_solve(k2, f, **opts):
    """Functional form of HelmholtzSolve."""
    return HelmholtzSolve.apply(k2, f, opts)
