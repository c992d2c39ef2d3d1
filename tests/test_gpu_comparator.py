"""GPU parity of the fixed-shift comparator (Sec. 2.2, Table 3's MG-FGMRES:
the cycle built on -Delta - (1 + i beta) k^2 on every level, including the
finest, preconditioning the unshifted problem), with both smoothers, in
GMRES/FGMRES and in the standalone refinement form u <- u + M (f - A u).
Bars as in the other parity tests (histories element-wise up to where the
oracle's own runs part, solutions against the oracle's drift)."""

import numpy as np
import pytest

from oracle import cycle as C
from oracle import helmholtz as H
from oracle import krylov as K
from paper_1211_4752_amd import workloads as W
from test_gpu_parity import _compare_hist, check_gmres
from test_gpu_smoother import check_fgmres

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BETA = 0.5


def _setup(wl, smoother, precision="c128"):
    from paper_1211_4752_amd import mg
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = len(wl.n)
    prob = H.Problem(wl.n, wl.h, wl.k2, (wl.ecs,) * d, (wl.ecs,) * d, wl.ecs_angle)
    L = H.auto_levels(prob.n)
    sig = np.full(L, 1 + 1j * BETA)
    levels = H.build_hierarchy(prob, sigma=sig)
    k2 = torch.tensor(wl.k2, dtype=torch.float64, device="cuda:0")
    s = mg.Solver(wl.n, wl.h, k2, ecs=wl.ecs, ecs_angle=wl.ecs_angle, sigma=sig, nrhs=wl.f.shape[0],
                  smoother=smoother, precision=precision)
    assert s.num_levels == L
    np.testing.assert_allclose(s.sigma(), sig, atol=1e-15)
    return s, levels, H.operator(prob)


def gpu(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.complex128, device="cuda:0")


@pytest.mark.parametrize("smoother", ["jacobi", "gmres3"])
def test_fixed_shift_krylov(smoother):
    wl = W.heterogeneous_2d(127, 2, ecs=4)
    s, levels, A = _setup(wl, smoother)
    vc = C.VCycle(levels, smoother="gmres" if smoother == "gmres3" else "jacobi")
    u = s.empty()
    status, its, hists = s.solve(u, gpu(wl.f), mode="gmres", rtol=1e-8, maxit=2000, restart=20)
    assert status == "converged"
    got = u.cpu().numpy()
    for r in range(2):
        if smoother == "gmres3":
            it = check_fgmres(got[r].ravel(), hists[r], its[r], A, vc.precondition, wl.f[r].ravel(), 1e-8, 2000)
        else:
            it = check_gmres(got[r].ravel(), hists[r], its[r], A, vc.precondition, wl.f[r].ravel(), 1e-8, 2000)
        print("fixed shift", smoother, r, "oracle", it, "gpu", its[r], flush=True)
        true = np.linalg.norm(wl.f[r].ravel() - A @ got[r].ravel()) / np.linalg.norm(wl.f[r])
        assert true <= 1e-8 * (1 + 1e-6)
    s.close()


def test_fixed_shift_standalone_refinement():
    wl = W.constant_2d(127, 0.3, ecs=16)
    s, levels, A = _setup(wl, "gmres3")
    vc = C.VCycle(levels, smoother="gmres")
    u = s.empty()
    status, its, hists = s.solve(u, gpu(wl.f), mode="standalone", rtol=1e-6, maxit=60)
    uo, ho, ito, sto = K.refine_standalone(A, vc.precondition, wl.f[0].ravel(), rtol=1e-6, maxit=60)
    print("fixed shift standalone", status, its, sto, ito, flush=True)
    _compare_hist(hists[0], ho, 1e-8)
    assert its[0] == ito
    s.close()


def test_fixed_shift_mixed():
    wl = W.heterogeneous_2d(127, 1, ecs=4)
    s, levels, A = _setup(wl, "gmres3", precision="mixed")
    u = s.empty()
    status, its, hists = s.solve(u, gpu(wl.f), mode="gmres", rtol=1e-10, maxit=2000, restart=20)
    assert status == "converged"
    import scipy.sparse.linalg as spla
    exact = spla.spsolve(A.tocsc(), wl.f[0].ravel())
    err = np.linalg.norm(u[0].cpu().numpy().ravel() - exact) / np.linalg.norm(exact)
    print("fixed shift mixed", its, err, flush=True)
    assert err <= 1e-6
    s.close()
