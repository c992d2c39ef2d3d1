"""Discretisation of the shifted Helmholtz operator and its level hierarchy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

What is computed, and where the paper fixes it
----------------------------------------------
* The discrete problem (-Delta^h - k^2) u = chi on a uniform vertex-centred
  grid with homogeneous Dirichlet ghosts (Sec. 2, eq. HH).
* Exterior complex scaling (ECS) absorbing layers: the grid is mapped onto a
  complex contour near the boundary (Sec. 2.4 and the constant-k model of
  Sec. 4.1).  The paper gives neither the contour nor the discretisation; the
  reading used here (documented as a design reading) is the piecewise map
  Z(x) = x inside [a, b], a + (x - a) e^{i phi} left of a, b + (x - b) e^{i phi}
  right of b, discretised by the standard non-uniform 3-point formula for
  -d^2/dz^2 on the mapped nodes.  With phi = 0 it is the uniform stencil.
* The level-dependent operators of Sec. 3.1 (eq. cslvariant): on level l the
  operator is -Delta^{h_l} - sigma_l k^2 with h_l = 2^l h_0, sigma_0 = 1.
* The shift schedule theta_l = l * theta_max / p, p = number of levels
  (Sec. 3.1, the paragraph after eq. csgvariant).
* Coarse operators by rediscretisation (Sec. 2); k^2 on coarse grids is
  sampled at the coarse nodes (injection).

Parity: every function here is pinned by tests/test_oracle_discretisation.py
(closed-form Dirichlet eigenpairs, manufactured solution, ECS identities,
printed d-theta values).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


# ---------------------------------------------------------------------------
# 1D coefficients
# ---------------------------------------------------------------------------

def ecs_nodes(n: int, h: float, length: float, ecs_lo: float, ecs_hi: float,
              phi: float) -> np.ndarray:
    """Complex node coordinates z_j = Z(j h), j = 0 .. n+1 (Sec. 2.4 reading).

    ``length`` is the physical extent (n+1) h, ``ecs_lo`` / ``ecs_hi`` the
    physical widths of the complex-scaled layers at each end (0 = none).
    The layer starts at a = ecs_lo and ends at b = length - ecs_hi.
    """
    x = h * np.arange(n + 2, dtype=np.float64)
    a = ecs_lo
    b = length - ecs_hi
    rot = np.exp(1j * phi)
    z = x.astype(np.complex128)
    left = x < a
    right = x > b
    z[left] = a + (x[left] - a) * rot
    z[right] = b + (x[right] - b) * rot
    return z


def axis_coefficients(z: np.ndarray):
    """3-point coefficients (c_minus, c_zero, c_plus) of -d^2/dz^2.

    For interior node j (1..n) with spacings hm = z_j - z_{j-1} and
    hp = z_{j+1} - z_j the second difference on non-uniform nodes gives
        c_minus = -2 / ((hm + hp) hm),  c_plus = -2 / ((hm + hp) hp),
        c_zero  = -(c_minus + c_plus),
    which is (-1, 2, -1) / h^2 on a uniform grid (Sec. 2, eq. HH).
    Returns three complex arrays of length n (index 0 <-> node 1).
    """
    hm = z[1:-1] - z[:-2]
    hp = z[2:] - z[1:-1]
    cm = -2.0 / ((hm + hp) * hm)
    cp = -2.0 / ((hm + hp) * hp)
    c0 = -(cm + cp)
    return cm, c0, cp


def axis_matrix(cm, c0, cp) -> sp.csr_matrix:
    """Tridiagonal n x n matrix of one axis with Dirichlet ghosts dropped."""
    n = len(c0)
    return sp.diags([cm[1:], c0, cp[:-1]], [-1, 0, 1], shape=(n, n),
                    format="csr", dtype=np.complex128)


def axis_weights(z: np.ndarray) -> np.ndarray:
    """Diagonal W_j = (hm + hp) / 2 that symmetrises one axis matrix (Sec. 2.4 reading)."""
    return 0.5 * (z[2:] - z[:-2])


# ---------------------------------------------------------------------------
# Operators on a d-dimensional tensor grid, x fastest
# ---------------------------------------------------------------------------

def laplacian(axis_mats) -> sp.csr_matrix:
    """Sum over axes of I (x) ... (x) T_axis (x) ... (x) I.

    ``axis_mats[0]`` is the x axis (fastest varying index).  The flat index of
    point (i_x, i_y, i_z) is i_x + n_x (i_y + n_y i_z), so the x factor is the
    rightmost Kronecker factor.
    """
    d = len(axis_mats)
    sizes = [m.shape[0] for m in axis_mats]
    total = None
    for a in range(d):
        term = None
        for b in reversed(range(d)):          # slowest axis first
            f = axis_mats[a] if b == a else sp.identity(sizes[b], format="csr",
                                                       dtype=np.complex128)
            term = f if term is None else sp.kron(term, f, format="csr")
        total = term if total is None else total + term
    return total.tocsr()


def shifted_operator(axis_mats, k2: np.ndarray, sigma: complex) -> sp.csr_matrix:
    """A~ = -Delta^h - sigma k^2 (Sec. 3.1, eq. cslvariant)."""
    lap = laplacian(axis_mats)
    return (lap - sp.diags(sigma * k2.ravel().astype(np.complex128))).tocsr()


# ---------------------------------------------------------------------------
# Shift schedule (Sec. 3.1)
# ---------------------------------------------------------------------------

def theta_schedule(nlevels: int, theta_max: float = math.pi / 6) -> np.ndarray:
    """theta_l = l * dtheta, dtheta = theta_max / p with p = nlevels (Sec. 3.1)."""
    return np.arange(nlevels) * (theta_max / nlevels)


def sigma_schedule(nlevels: int, theta_max: float = math.pi / 6,
                   kind: str = "exp") -> np.ndarray:
    """Per-level shift sigma_l multiplying k^2 (Sec. 3.1, eq. cslvariant).

    kind="exp":  sigma_l = e^{i theta_l} (the paper's form with r = 1).
    kind="beta": sigma_l = 1 + i tan(theta_l), the (1 + beta i) form of
                 Sec. 2.2 / 2.3 that the paper relates to r = 1/cos(theta).
    """
    th = theta_schedule(nlevels, theta_max)
    if kind == "exp":
        return np.exp(1j * th)
    if kind == "beta":
        return 1.0 + 1j * np.tan(th)
    raise ValueError(kind)


# ---------------------------------------------------------------------------
# Level hierarchy
# ---------------------------------------------------------------------------

def coarse_size(n: int) -> int:
    """n_{l+1} = (n_l - 1) / 2 interior points: coarse I <-> fine 2I+1 (Sec. 2.1)."""
    return (n - 1) // 2


def auto_levels(n) -> int:
    """Coarsen while every axis is odd and the next size is at least 2."""
    n = list(n)
    levels = 1
    while all(m % 2 == 1 and coarse_size(m) >= 2 for m in n):
        n = [coarse_size(m) for m in n]
        levels += 1
    return levels


def inject_k2(k2: np.ndarray) -> np.ndarray:
    """Coarse k^2 sampled at the coarse nodes: k2_c[I] = k2_f[2I+1] per axis."""
    sl = tuple(slice(1, None, 2) for _ in range(k2.ndim))
    c = k2[sl]          # odd indices 1, 3, ...; trim in case an axis is even
    trim = tuple(slice(0, coarse_size(m)) for m in k2.shape)
    return np.ascontiguousarray(c[trim])


@dataclass
class Level:
    n: tuple          # interior points per axis, x first
    h: tuple          # grid spacing per axis
    sigma: complex    # shift multiplying k^2 on this level
    k2: np.ndarray    # real, array shape (n_z, n_y, n_x) / (n_y, n_x)
    coef: list        # per axis (cm, c0, cp)
    weights: list     # per axis symmetrising diagonal
    A: sp.csr_matrix = field(repr=False, default=None)

    @property
    def size(self) -> int:
        return int(np.prod(self.n))

    def diagonal(self) -> np.ndarray:
        return self.A.diagonal()


@dataclass
class Problem:
    """Inputs that define one discrete problem (Sec. 2, eq. HH; Sec. 4)."""
    n: tuple                  # interior points per axis, x first
    h: tuple                  # spacing per axis
    k2: np.ndarray            # array shaped (n_z, n_y, n_x) or (n_y, n_x)
    ecs_lo: tuple = None      # complex-scaled cells at the low end of each axis
    ecs_hi: tuple = None      # ... and at the high end
    ecs_angle: float = math.pi / 4


def build_hierarchy(prob: Problem, sigma: np.ndarray | None = None,
                    nlevels: int | None = None, theta_max: float = math.pi / 6
                    ) -> list:
    """Rediscretised level hierarchy with per-level shifts (Sec. 3.1)."""
    d = len(prob.n)
    if nlevels is None or nlevels == 0:
        nlevels = auto_levels(prob.n)
    if sigma is None:
        sigma = sigma_schedule(nlevels, theta_max)
    sigma = np.asarray(sigma, dtype=np.complex128)
    assert len(sigma) >= nlevels
    ecs_lo = prob.ecs_lo or (0,) * d
    ecs_hi = prob.ecs_hi or (0,) * d
    lengths = [(prob.n[a] + 1) * prob.h[a] for a in range(d)]
    widths_lo = [ecs_lo[a] * prob.h[a] for a in range(d)]
    widths_hi = [ecs_hi[a] * prob.h[a] for a in range(d)]

    levels = []
    n = list(prob.n)
    h = list(prob.h)
    k2 = np.asarray(prob.k2, dtype=np.float64)
    for l in range(nlevels):
        coef, wts, mats = [], [], []
        for a in range(d):
            z = ecs_nodes(n[a], h[a], lengths[a], widths_lo[a], widths_hi[a],
                          prob.ecs_angle)
            cm, c0, cp = axis_coefficients(z)
            coef.append((cm, c0, cp))
            wts.append(axis_weights(z))
            mats.append(axis_matrix(cm, c0, cp))
        A = shifted_operator(mats, k2, complex(sigma[l]))
        levels.append(Level(tuple(n), tuple(h), complex(sigma[l]), k2, coef,
                            wts, A))
        if l + 1 < nlevels:
            n = [coarse_size(m) for m in n]
            h = [2.0 * x for x in h]
            k2 = inject_k2(k2)
    return levels


def operator(prob: Problem, sigma: complex = 1.0) -> sp.csr_matrix:
    """The finest-grid operator -Delta^h - sigma k^2 alone."""
    return build_hierarchy(prob, sigma=np.array([sigma]), nlevels=1)[0].A
