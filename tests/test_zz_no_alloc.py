"""GPU: mg_cycle_noalloc (the cycle for callers that cannot allocate, with
the library's fixed per-GPU scratch) against mg_cycle through the C ABI.

Both run the same recorded kernels on the same inputs, so the results and
the incoming residual norms must be equal bit for bit.  Two calls in a row
share the scratch, the second on a smaller problem, for both smoothers and
both precisions, plus a 3D pair; the first output is also held to the
oracle's cycle at the bars of the parity tests.
"""

import numpy as np
import pytest

from oracle import cycle as C
from oracle import helmholtz as H
from paper_1211_4752_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def rnd(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def run_pair(s, wl, seed):
    dev = _dev()
    shape = (wl.f.shape[0],) + tuple(reversed(wl.n))
    u0 = rnd(shape, seed)
    f = torch.tensor(rnd(shape, seed + 1), dtype=torch.complex128, device=dev)
    ua = torch.tensor(u0, dtype=torch.complex128, device=dev)
    ra = s.cycle(ua, f, residual=True)
    ub = torch.tensor(u0, dtype=torch.complex128, device=dev)
    rb = s.cycle_noalloc(ub, f, residual=True)
    torch.cuda.synchronize()
    print("noalloc", wl.n, s.smoother, s.precision, "max |diff|", float((ua - ub).abs().max()), flush=True)
    assert torch.equal(ua, ub)
    assert np.array_equal(ra, rb)
    return u0, f.cpu().numpy(), ub.cpu().numpy()


@pytest.mark.parametrize("smoother", ["jacobi", "gmres3"])
@pytest.mark.parametrize("precision", ["c128", "mixed"])
def test_noalloc_equals_cycle(smoother, precision):
    from paper_1211_4752_amd import mg
    mg.lib()
    dev = _dev()
    wls = [W.heterogeneous_2d(127, 2, ecs=4), W.heterogeneous_2d(63, 1, ecs=2)]   # second call smaller
    for i, wl in enumerate(wls):
        s = mg.Solver(wl.n, wl.h, torch.tensor(wl.k2, dtype=torch.float64, device=dev), ecs=wl.ecs,
                      ecs_angle=wl.ecs_angle, theta_max=wl.theta_max, nrhs=wl.f.shape[0], smoother=smoother,
                      precision=precision)
        u0, f, got = run_pair(s, wl, 10 + i)
        s.close()
        if i == 0 and precision == "c128":
            d = len(wl.n)
            levels = H.build_hierarchy(H.Problem(wl.n, wl.h, wl.k2, (wl.ecs,) * d, (wl.ecs,) * d, wl.ecs_angle))
            vc = C.VCycle(levels, smoother="gmres" if smoother == "gmres3" else "jacobi")
            for r in range(u0.shape[0]):
                want = vc(u0[r].ravel(), f[r].ravel())
                err = np.abs(got[r].ravel() - want).max() / np.abs(want).max()
                assert err < (1e-10 if smoother == "gmres3" else 1e-11), err


def test_noalloc_3d():
    from paper_1211_4752_amd import mg
    dev = _dev()
    for i, wl in enumerate([W.constant_3d(31, 0.5, 2), W.constant_3d(15, 0.5, 1)]):
        s = mg.Solver(wl.n, wl.h, torch.tensor(wl.k2, dtype=torch.float64, device=dev), ecs=wl.ecs,
                      ecs_angle=wl.ecs_angle, theta_max=wl.theta_max, nrhs=1, smoother="gmres3")
        run_pair(s, wl, 20 + i)
        s.close()


def test_noalloc_rejects_oversize():
    """A context whose work space exceeds the fixed scratch gets MG_E_INVAL
    (1023^2 x 16 right-hand sides, complex128) and leaves u untouched."""
    from paper_1211_4752_amd import mg
    dev = _dev()
    n = 1023
    k2 = torch.full((n, n), 100.0, dtype=torch.float64, device=dev)
    s = mg.Solver((n, n), 1.0 / (n + 1), k2, nrhs=16)
    u = s.empty()
    f = torch.ones_like(u)
    with pytest.raises(mg.MGError) as e:
        s.cycle_noalloc(u, f)
    assert e.value.status == mg.MG_E_INVAL
    assert float(u.abs().max()) == 0.0
    s.close()
