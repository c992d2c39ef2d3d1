"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws inputs (wavenumber fields, point sources, receiver
positions, problem sizes).  It holds none of the method's arithmetic and is
shared by the GPU path's tests/benchmark and by the CPU oracle's tests.

Shapes follow the paper's constant-k model (Sec. 4.1: unit square, centre
point source, absorbing layer) extended with a smooth heterogeneous medium:

* ``grf``: a zero-mean Gaussian random field with Gaussian covariance
  exp(-r^2 / (2 ell^2)), made by filtering seeded white noise in Fourier space
  on a zero-padded periodic grid of 2(n+1) points per axis, cropped to the
  n^d interior nodes, scaled to unit sample standard deviation.
* ``heterogeneous_k2``: k = k0 (1 + amp g), g = clip(grf, -1, 1),
  k0 chosen so that max(k) h equals a target kh (0.625: ten points per
  wavelength, Sec. 4.1).  Returns k^2 (the operator takes k^2).
* point sources at seeded uniform interior nodes inside the physical region;
  unit value, no 1/h^d scaling (Sec. 4.1).

Arrays are NumPy float64 / complex128 shaped (n_z, n_y, n_x) or (n_y, n_x),
i.e. x fastest.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def grf(n: int, dim: int, ell: float, seed: int) -> np.ndarray:
    """Unit-variance Gaussian random field on the n^dim interior nodes of the
    unit cube, correlation length ell (Gaussian covariance)."""
    rng = np.random.default_rng(seed)
    h = 1.0 / (n + 1)
    m = 2 * (n + 1)
    noise = rng.standard_normal((m,) * dim)
    freqs = np.fft.fftfreq(m, d=h)
    grids = np.meshgrid(*([freqs] * dim), indexing="ij")
    xi2 = sum(g * g for g in grids)
    # the spectral density of exp(-r^2/(2 ell^2)) is proportional to
    # exp(-2 pi^2 ell^2 |xi|^2); filter with its square root
    filt = np.exp(-math.pi ** 2 * ell ** 2 * xi2)
    field = np.real(np.fft.ifftn(np.fft.fftn(noise) * filt))
    crop = field[(slice(0, n),) * dim]
    crop = crop - crop.mean()
    return crop / crop.std()


def heterogeneous_k2(n: int, dim: int, seed: int, amp: float = 0.3,
                     ell: float = 0.1, kh_max: float = 0.625) -> np.ndarray:
    """k^2 of k = k0 (1 + amp clip(grf, -1, 1)) with max(k) h = kh_max."""
    h = 1.0 / (n + 1)
    g = np.clip(grf(n, dim, ell, seed), -1.0, 1.0)
    shape = 1.0 + amp * g
    k0 = kh_max / (h * shape.max())
    return (k0 * shape) ** 2


def perturbed_k2(k2: np.ndarray, seed: int, amp: float = 0.05,
                 ell: float = 0.1) -> np.ndarray:
    """k_true = k (1 + amp g2), g2 an independent field (adjoint workload)."""
    n = k2.shape[-1]
    g2 = np.clip(grf(n, k2.ndim, ell, seed), -1.0, 1.0)
    return k2 * (1.0 + amp * g2) ** 2


def constant_k2(n: int, dim: int, k: float) -> np.ndarray:
    return np.full((n,) * dim, float(k) ** 2)


def source_nodes(n: int, dim: int, count: int, seed: int, lo: int, hi: int,
                 max_y: int | None = None) -> np.ndarray:
    """``count`` distinct interior nodes, each coordinate uniform in [lo, hi].

    Rows are (i_x, i_y[, i_z]).  ``max_y`` optionally bounds i_y from above.
    """
    rng = np.random.default_rng(seed)
    out, seen = [], set()
    while len(out) < count:
        p = tuple(int(v) for v in rng.integers(lo, hi + 1, size=dim))
        if max_y is not None and p[1] > max_y:
            continue
        if p not in seen:
            seen.add(p)
            out.append(p)
    return np.array(out, dtype=np.int64)


def point_sources(n, nodes) -> np.ndarray:
    """Stack of unit point-source right-hand sides, shape (count, *grid)."""
    n = tuple(n)                          # x first
    dim = len(n)
    shape = tuple(reversed(n))            # array order: slowest first
    f = np.zeros((len(nodes),) + shape, dtype=np.complex128)
    for s, p in enumerate(nodes):
        f[(s,) + tuple(reversed(tuple(int(v) for v in p[:dim])))] = 1.0
    return f


def centre_source(n) -> np.ndarray:
    """Unit source at the centre node (n-1)/2 of every axis (Sec. 4.1)."""
    n = tuple(n)
    return point_sources(n, [tuple((m - 1) // 2 for m in n)])[0]


def receiver_nodes(n: int, count: int = 128, row: int = 460) -> np.ndarray:
    """Nodes on the line i_y = row nearest x = 1/32 + (r + 1/2) (15/16) / count."""
    h = 1.0 / (n + 1)
    xs = 1.0 / 32 + (np.arange(count) + 0.5) * (15.0 / 16.0) / count
    ix = np.rint(xs / h).astype(np.int64) - 1          # interior index of node
    return np.stack([ix, np.full(count, row, dtype=np.int64)], axis=1)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    n: tuple              # interior points per axis, x first
    k2: np.ndarray        # shaped like the grid, slowest axis first
    f: np.ndarray         # (nrhs, *grid) complex128
    ecs: int              # complex-scaled cells on every side (0 = Dirichlet)
    ecs_angle: float = math.pi / 4
    theta_max: float = math.pi / 6
    spacing: tuple | None = None   # grid spacing per axis (None: 1/(n+1))
    sides: tuple | None = None     # ((lo per axis), (hi per axis)) ECS cells,
                                   # overriding ``ecs`` when set

    @property
    def h(self):
        if self.spacing is not None:
            return tuple(self.spacing)
        return tuple(1.0 / (m + 1) for m in self.n)

    @property
    def ecs_lo(self):
        return tuple(self.sides[0]) if self.sides else (self.ecs,) * len(self.n)

    @property
    def ecs_hi(self):
        return tuple(self.sides[1]) if self.sides else (self.ecs,) * len(self.n)

    @property
    def dofs(self) -> int:
        return int(np.prod(self.n)) * self.f.shape[0]


def dirichlet_constant_2d(n: int = 63, k: float = 40.0) -> Workload:
    """Constant k, homogeneous Dirichlet, centre source (63^2, k = 40)."""
    return Workload("dirichlet_const_2d_%d" % n, (n, n), constant_k2(n, 2, k),
                    centre_source((n, n))[None], ecs=0)


def heterogeneous_2d(n: int = 1023, nrhs: int = 8, ecs: int | None = None,
                     field_seed: int = 2, source_seed: int = 3) -> Workload:
    """GRF medium (+-30 %, ell = 0.1, max kh = 0.625), ECS layer of
    (n+1)/32 cells, ``nrhs`` unit sources in the physical region."""
    if ecs is None:
        ecs = (n + 1) // 32
    k2 = heterogeneous_k2(n, 2, field_seed)
    nodes = source_nodes(n, 2, nrhs, source_seed, ecs, n - 1 - ecs)
    return Workload("grf_2d_%d_x%d" % (n, nrhs), (n, n), k2,
                    point_sources((n, n), nodes), ecs=ecs)


def constant_3d(n: int = 255, kh: float = 0.5, ecs: int = 16) -> Workload:
    """Constant k with k h = kh, 7-point, ECS layer, centre source."""
    k = kh * (n + 1)
    return Workload("const_3d_%d" % n, (n, n, n), constant_k2(n, 3, k),
                    centre_source((n, n, n))[None], ecs=ecs)


def constant_2d(n: int, kh: float, ecs: int | None = None) -> Workload:
    if ecs is None:
        ecs = (n + 1) // 32
    k = kh * (n + 1)
    return Workload("const_2d_%d" % n, (n, n), constant_k2(n, 2, k),
                    centre_source((n, n))[None], ecs=ecs)


UNEVEN_SIZES = sorted({m * 2 ** q - 1 for m in (4, 5, 6, 7) for q in range(3, 9)
                       if 127 <= m * 2 ** q - 1 <= 1023})


def uneven_batch(count: int = 24, seed: int = 5):
    """Sizes drawn with replacement from {m 2^q - 1 in [127, 1023], m = 4..7}
    and a constant kh ~ U[0.3, 0.625] each; centre source; ECS (n+1)/32."""
    rng = np.random.default_rng(seed)
    sizes = rng.choice(UNEVEN_SIZES, size=count, replace=True)
    khs = rng.uniform(0.3, 0.625, size=count)
    return [constant_2d(int(n), float(kh)) for n, kh in zip(sizes, khs)]


def batched_2d(n: int = 511, nrhs: int = 64, count: int = 24):
    """Batched workload: ``nrhs`` unit sources (seed 4) on one n^2 GRF
    medium as in heterogeneous_2d, plus ``count`` uneven constant-kh
    problems (uneven_batch)."""
    return [heterogeneous_2d(n, nrhs, source_seed=4)] + uneven_batch(count)



# ---------------------------------------------------------------------------
# Analytic models of Sec. 4.2 and 4.3
# ---------------------------------------------------------------------------
#
# The grid holds the physical region plus the complex-scaled layers, as for
# the unit-square workloads.  The paper gives the physical grid (its n_x x
# n_y cells over Omega) but not the layers, so the physical spacing is kept
# and layers are added outside Omega: a quarter of the x cell count on every
# outgoing side, which makes every axis m 2^q - 1 interior points with
# m in {3, 5}.  Coefficients inside a layer are the model's own formula
# evaluated at the layer node's real coordinate (the wedge clamps the
# coordinate into Omega first: its velocity is only defined there).

WEDGE_X, WEDGE_Y = 600.0, 1000.0


def wedge_velocity(x, y):
    """Piecewise-constant velocity c(x, y) of the wedge model (Sec. 4.2):
    2000 below the line y = x/6 + 400, 1500 between it and y = 800 - x/3,
    3000 above."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return np.where(y < x / 6.0 + 400.0, 2000.0,
                    np.where(y < -x / 3.0 + 800.0, 1500.0, 3000.0))


def _axis(cells: int, layer_lo: int, layer_hi: int, length: float):
    """Interior-node count, spacing and the physical coordinate of every
    interior node of an axis of ``cells`` physical cells over (0, length)
    with ``layer_lo`` / ``layer_hi`` extra cells outside it."""
    h = length / cells
    n = cells + layer_lo + layer_hi - 1
    x = (np.arange(n) + 1 - layer_lo) * h
    return n, h, x


def wedge_2d(f_hz: float, cells_x: int) -> Workload:
    """2D wedge model (Sec. 4.2, Table 6): Omega = (0,600) x (0,1000) on
    cells_x x 2 cells_x physical cells, k^2 = (2 pi f / c)^2, unit point
    source at (300, 0), ECS layers of cells_x / 4 cells on all four sides."""
    L = cells_x // 4
    nx, hx, x = _axis(cells_x, L, L, WEDGE_X)
    ny, hy, y = _axis(2 * cells_x, L, L, WEDGE_Y)
    X, Y = np.meshgrid(np.clip(x, 0, WEDGE_X), np.clip(y, 0, WEDGE_Y))
    k2 = (2.0 * math.pi * f_hz / wedge_velocity(X, Y)) ** 2
    src = (int(round(300.0 / hx)) + L - 1, L - 1)       # node at (300, 0)
    return Workload("wedge_2d_%dhz_%dx%d" % (round(f_hz), cells_x, 2 * cells_x), (nx, ny), k2,
                    point_sources((nx, ny), [src]), ecs=L, spacing=(hx, hy),
                    sides=((L, L), (L, L)))


def wedge_3d(f_hz: float, cells_x: int = 64) -> Workload:
    """3D wedge model (Sec. 4.2, Table 7): the third axis z repeats the x
    axis (0, 600) and the velocity does not depend on z; unit source at
    (300, 0, 300); layers of cells_x / 4 cells on all six sides."""
    L = cells_x // 4
    nx, hx, x = _axis(cells_x, L, L, WEDGE_X)
    ny, hy, y = _axis(2 * cells_x, L, L, WEDGE_Y)
    X, Y = np.meshgrid(np.clip(x, 0, WEDGE_X), np.clip(y, 0, WEDGE_Y))
    k2_xy = (2.0 * math.pi * f_hz / wedge_velocity(X, Y)) ** 2
    k2 = np.ascontiguousarray(np.broadcast_to(k2_xy, (nx, ny, nx)))
    c = int(round(300.0 / hx)) + L - 1
    return Workload("wedge_3d_%dhz_%dx%dx%d" % (round(f_hz), cells_x, 2 * cells_x, cells_x),
                    (nx, ny, nx), k2, point_sources((nx, ny, nx), [(c, L - 1, c)]), ecs=L,
                    spacing=(hx, hy, hx), sides=((L,) * 3, (L,) * 3))


IONIZATION_R = 50.0


def ionization_2d(k0: float, cells: int) -> Workload:
    """Quantum-mechanical ionization model (Sec. 4.3, Table 8): Omega =
    (0, 50)^2 on cells^2 physical cells, k^2(x, y) = exp(-x^2) + exp(-y^2)
    + k0^2, right-hand side chi = exp(-(x^2 + y^2)) at the nodes, u = 0 on
    x = 0 and y = 0 (no layer there), ECS layers of cells / 4 cells beyond
    x = 50 and y = 50."""
    L = cells // 4
    n, h, x = _axis(cells, 0, L, IONIZATION_R)
    X, Y = np.meshgrid(x, x)
    k2 = np.exp(-X * X) + np.exp(-Y * Y) + float(k0) ** 2
    f = np.exp(-(X * X + Y * Y)).astype(np.complex128)[None]
    return Workload("ionization_2d_k%g_%d" % (k0, cells), (n, n), k2, f, ecs=L,
                    spacing=(h, h), sides=((0, 0), (L, L)))


# (f, physical cells in x) of Table 6, f of Table 7 and (k0, cells) of Table 8
WEDGE_2D_TABLE6 = [(10, 64), (20, 128), (30, 128), (40, 256), (50, 256)]
WEDGE_3D_TABLE7 = [12, 14, 16, 18, 20]
IONIZATION_TABLE8 = [(1, 128), (2, 256), (3, 256), (4, 512), (5, 512)]
