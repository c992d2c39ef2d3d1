"""GPU checks at the full sizes of the 3D and adjoint workloads.

* 3D: 255^3 interior grid, constant k with k h = 0.5, ECS layer of 16 cells,
  centre source, GMRES(3)-smoothed cycle in FGMRES(20), solved to 1e-10 in
  FP64 and in mixed precision (complex64 cycle).  Checks: the residual of
  both solutions under the oracle's own sparse operator, and the stated
  error of the mixed solution against the FP64 one (at most 1e-6 relative).
  The cycle itself is held to the oracle at 31^3 .. 63^3 in the parity tests;
  the oracle cannot run a solve at this size in a test's time.
* Adjoint: 511^2 heterogeneous medium, 16 sources, 128 receivers on the
  row y = 0.9, loss 0.5 sum ||P u - d||^2 with data from a perturbed medium;
  dL/d(k^2) through torch.autograd (forward and adjoint GMRES(3)-smoothed
  FGMRES solves to 1e-10) against the oracle's gradient from LU-factorised
  exact solves, and against Sherman-Morrison central differences at 32
  seeded points (both 1e-6 relative).
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import adjoint as AD
from oracle import helmholtz as H
from paper_1211_4752_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)


def test_3d_255_fp64_and_mixed():
    from paper_1211_4752_amd import mg
    dev = _dev()
    wl = W.constant_3d(255, 0.5, 16)
    k2 = torch.tensor(wl.k2, dtype=torch.float64, device=dev)
    f = torch.tensor(wl.f, dtype=torch.complex128, device=dev)
    sols = {}
    for prec in ("c128", "mixed"):
        s = mg.Solver(wl.n, wl.h, k2, ecs=wl.ecs, ecs_angle=wl.ecs_angle, theta_max=wl.theta_max, nrhs=1,
                      precision=prec, smoother="gmres3")
        u = s.empty()
        st, its, hists = s.solve(u, f, mode="gmres", rtol=1e-10, maxit=600, restart=20)
        say("3d 255", prec, st, its)
        assert st == "converged"
        sols[prec] = u.cpu().numpy().ravel()
        s.close()
        del u
    A = H.operator(H.Problem(wl.n, wl.h, wl.k2, (wl.ecs,) * 3, (wl.ecs,) * 3, wl.ecs_angle))
    fv = wl.f[0].ravel()
    for prec, x in sols.items():
        res = np.linalg.norm(fv - A @ x) / np.linalg.norm(fv)
        say("oracle residual", prec, res)
        assert res <= 1e-10 * (1 + 1e-6)
    err = np.linalg.norm(sols["mixed"] - sols["c128"]) / np.linalg.norm(sols["c128"])
    say("mixed vs fp64 error", err)
    assert err <= 1e-6


def test_adjoint_gradient_511():
    from paper_1211_4752_amd.autograd import helmholtz_solve
    dev = _dev()
    n, nshots, nrec = 511, 16, 128
    ecs = (n + 1) // 32
    k2 = W.heterogeneous_k2(n, 2, seed=2)
    k2_true = W.perturbed_k2(k2, seed=7)
    nodes = W.source_nodes(n, 2, nshots, seed=6, lo=ecs, hi=n - 1 - ecs, max_y=int(0.8 * (n + 1)))
    f = W.point_sources((n, n), nodes)
    rec = W.receiver_nodes(n, nrec, 460)
    idx = rec[:, 1] * n + rec[:, 0]
    P = sp.csr_matrix((np.ones(len(idx)), (np.arange(len(idx)), idx)), shape=(len(idx), n * n))

    def prob(kk):
        return H.Problem((n, n), (1.0 / (n + 1),) * 2, kk, (ecs, ecs), (ecs, ecs), math.pi / 4)

    lu_true = spla.splu(H.operator(prob(k2_true)).tocsc())
    d = np.stack([P @ lu_true.solve(f[s].ravel()) for s in range(nshots)])
    del lu_true
    k2_t = torch.tensor(k2, dtype=torch.float64, device=dev, requires_grad=True)
    u = helmholtz_solve(k2_t, torch.tensor(f, dtype=torch.complex128, device=dev), n=(n, n), h=1.0 / (n + 1),
                        ecs=ecs, rtol=1e-10, maxit=5000)
    Pt = torch.tensor(P.toarray(), dtype=torch.complex128, device=dev)
    loss = 0.5 * (u.reshape(nshots, -1) @ Pt.T - torch.tensor(d, device=dev)).abs().pow(2).sum()
    loss.backward()
    g_gpu = k2_t.grad.cpu().numpy().ravel()
    A = H.operator(prob(k2)).tocsc()
    lu = spla.splu(A)
    luh = spla.splu(A.conj().T.tocsc())
    us = [lu.solve(f[s].ravel()) for s in range(nshots)]
    lams = [luh.solve(AD.receiver_grad_u(us[s], P, d[s])) for s in range(nshots)]
    g_or = AD.grad_k2(us, lams)
    assert float(loss.detach()) == pytest.approx(AD.receiver_loss(us, P, d), rel=1e-8)
    err = np.abs(g_gpu - g_or).max() / np.abs(g_or).max()
    say("511 gradient vs oracle", err)
    assert err < 1e-6
    rng = np.random.default_rng(8)
    inner = np.array([i for i in range(n * n) if ecs <= i % n < n - ecs and ecs <= i // n < n - ecs])
    pts = rng.choice(inner, 32, replace=False)
    worst = 0.0
    for i in pts:
        eps = 1e-4 * k2.ravel()[i]
        e = np.zeros(n * n, complex)
        e[i] = 1
        z = lu.solve(e)
        diff = 0.0
        for t in (eps, -eps):
            Lt = 0.0
            for s in range(nshots):
                delta = t * us[s][i] / (1 - t * z[i]) * z
                r = P @ us[s] - d[s]
                Pd = P @ delta
                Lt += float(np.real(np.vdot(r, Pd)) + 0.5 * np.linalg.norm(Pd) ** 2)
            diff += Lt if t > 0 else -Lt
        fd = diff / (2 * eps)
        worst = max(worst, abs(g_gpu[i] - fd) / np.abs(g_or).max())
        assert g_gpu[i] == pytest.approx(fd, rel=1e-6, abs=1e-6 * np.abs(g_or).max())
    say("511 gradient vs differences (max abs / max |g|)", worst)
