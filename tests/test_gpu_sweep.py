"""GPU: plane-sweep variants of the omega-Jacobi cycle kernels (shape ids
3-5), on grids whose every axis leaves ragged tiles and chunks: 3D 71 x 23 x
39 (two x tiles of 64, three y tiles of 8, chunks of 16 or 32 planes) and 2D
287 x 47 (two row segments of 256, chunks of 16 or 32 rows).

The sweeps serve the zero-guess kernels: the coarse levels of every cycle
and level 0 when the cycle preconditions GMRES or runs in complex64 on the
residual.  Checked against the oracle: one FP64 cycle from a random iterate
(1e-11 relative, max norm), GMRES histories and iterates (1e-8 and 1e-9),
and the complex64 cycle against the oracle's complex64 cycle (1e-4); and
the cycle bit for bit against the tiled kernels (shape 0).
"""

import numpy as np
import pytest

from oracle import cycle as C
from oracle import helmholtz as H
from oracle import krylov as K
from paper_1211_4752_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)


def rnd(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def gpu(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.complex128, device=_dev())


def ragged(n, seed):
    """k h = 0.4 on the longest axis, k^2 perturbed by up to 20 %, two
    random right-hand sides, ECS layer of 2 cells."""
    rng = np.random.default_rng(seed)
    k = 0.4 * (max(n) + 1)
    k2 = (k * k) * (1.0 + 0.2 * rng.random(tuple(reversed(n))))
    return W.Workload("ragged", tuple(n), k2, rnd((2,) + tuple(reversed(n)), seed + 1), ecs=2)


CASES = {"3d_71x23x39": lambda: ragged((71, 23, 39), 7), "2d_287x47": lambda: ragged((287, 47), 9)}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("precision", ["c128", "mixed"])
def test_sweep_shapes(case, precision):
    from paper_1211_4752_amd import mg
    wl = CASES[case]()
    d = len(wl.n)
    levels = H.build_hierarchy(H.Problem(wl.n, wl.h, wl.k2, (wl.ecs,) * d, (wl.ecs,) * d, wl.ecs_angle))
    vc = C.VCycle(levels, smoother="jacobi")
    vc32 = C.VCycle(levels, smoother="jacobi", dtype=np.complex64)
    s = mg.Solver(wl.n, wl.h, torch.tensor(wl.k2, dtype=torch.float64, device=_dev()), ecs=wl.ecs,
                  ecs_angle=wl.ecs_angle, theta_max=wl.theta_max, nrhs=2, smoother="jacobi", precision=precision)
    grid = (2,) + tuple(reversed(wl.n))
    u0, f = rnd(grid, 11), rnd(grid, 12)
    for l in range(s.num_levels):
        s.tile_shape(l, 0)
    u = gpu(u0)
    s.cycle(u, gpu(f))
    tiled = u.cpu().numpy()
    for shape in (3, 4, 5):
        say(case, precision, "shape", shape)
        for l in range(s.num_levels):
            assert s.tile_shape(l, shape) == shape
        u = gpu(u0)
        s.cycle(u, gpu(f))
        got = u.cpu().numpy()
        assert np.array_equal(got, tiled), shape   # same operations in the same order as the tiles
        for r in range(2):
            if precision == "c128":
                want, bar = vc(u0[r].ravel(), f[r].ravel()), 1e-11
            else:
                res = f[r].ravel() - levels[0].A @ u0[r].ravel()
                want, bar = u0[r].ravel() + vc32.precondition(res), 1e-4
            err = np.abs(got[r].ravel() - want).max() / np.abs(want).max()
            say("  cycle rhs", r, err)
            assert err < bar, (shape, r, err)
        if precision == "c128":
            u = s.empty()
            st, its, hists = s.solve(u, gpu(wl.f), mode="gmres", rtol=1e-8, maxit=60, restart=20)
            x, hist, it, _ = K.gmres(levels[0].A, vc.precondition, wl.f[0].ravel(), rtol=1e-8, restart=20,
                                     maxit=60)
            err = np.linalg.norm(u[0].cpu().numpy().ravel() - x) / np.linalg.norm(x)
            dh = max(abs(a - b) / b for a, b in zip(hists[0], hist))
            say("  gmres", its, it, err, dh)
            assert its[0] == it and err < 1e-9 and dh < 1e-8
    s.close()
