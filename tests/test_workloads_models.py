"""The analytic model inputs of Sec. 4.2 (wedge) and Sec. 4.3 (ionization)
against the definitions printed there: velocity regions, wavenumber and
source formulas, source position, Dirichlet / outgoing sides, the paper's
physical grids and the 10-points-per-wavelength criterion."""

import math

import numpy as np
import pytest

from oracle import helmholtz as H
from paper_1211_4752_amd import workloads as W


@pytest.mark.parametrize("x,y,c", [(300, 100, 2000), (0, 399.9, 2000), (0, 400, 1500),
                                   (100, 500, 1500), (600, 499.9, 2000), (600, 500, 1500), (600, 600, 3000),
                                   (0, 800, 3000), (500, 900, 3000), (300, 699.9, 1500), (300, 700, 3000),
                                   (300, 449.9, 2000), (300, 450, 1500)])
def test_wedge_velocity_regions(x, y, c):
    # 2000 below y = x/6 + 400, 1500 up to y = 800 - x/3 (the lines meet at
    # x = 800, outside Omega), 3000 above
    assert W.wedge_velocity(x, y) == c


def _coords(wl, axis):
    lo = wl.ecs_lo[axis]
    return (np.arange(wl.n[axis]) + 1 - lo) * wl.h[axis]


@pytest.mark.parametrize("f_hz,cells", W.WEDGE_2D_TABLE6)
def test_wedge_2d_grid_and_source(f_hz, cells):
    wl = W.wedge_2d(f_hz, cells)
    assert wl.h == (600.0 / cells, 1000.0 / (2 * cells))
    x, y = _coords(wl, 0), _coords(wl, 1)
    # Omega's corners are grid nodes; the layer adds cells/4 cells per side
    assert x[wl.ecs_lo[0] - 1] == 0 and x[wl.ecs_lo[0] - 1 + cells] == 600
    assert y[wl.ecs_lo[1] - 1] == 0 and y[wl.ecs_lo[1] - 1 + 2 * cells] == 1000
    assert wl.ecs_lo == wl.ecs_hi == (cells // 4,) * 2
    # unit point source at (300, 0)
    (iy, ix), = np.argwhere(wl.f[0] != 0)
    assert (x[ix], y[iy]) == (300.0, 0.0) and wl.f[0][iy, ix] == 1
    # k^2 = (2 pi f / c)^2 with c from the physical point (clamped in the layer)
    X, Y = np.meshgrid(np.clip(x, 0, 600), np.clip(y, 0, 1000))
    c = np.where(Y < X / 6 + 400, 2000.0, np.where(Y < 800 - X / 3, 1500.0, 3000.0))
    np.testing.assert_allclose(wl.k2, (2 * math.pi * f_hz / c) ** 2, rtol=1e-15)
    assert set(np.unique(c)) == {1500.0, 2000.0, 3000.0}
    # the paper's grids keep k h below 0.625 (at least 10 points per wavelength)
    assert math.sqrt(wl.k2.max()) * max(wl.h) < 0.625
    # every axis coarsens to the same depth (m 2^q - 1 points, m in {3, 5}),
    # down to 2 x 4 points
    assert H.auto_levels(wl.n) == int(math.log2(cells))


def test_wedge_3d_repeats_x():
    wl = W.wedge_3d(16, 32)
    assert wl.n[2] == wl.n[0] and wl.h[2] == wl.h[0]
    for z in (0, wl.n[2] // 2, wl.n[2] - 1):
        np.testing.assert_array_equal(wl.k2[z], wl.k2[0])
    np.testing.assert_allclose(wl.k2[0], W.wedge_2d(16, 32).k2, rtol=1e-15)
    (iz, iy, ix), = np.argwhere(wl.f[0] != 0)
    x, y, z = _coords(wl, 0), _coords(wl, 1), _coords(wl, 2)
    assert (x[ix], y[iy], z[iz]) == (300.0, 0.0, 300.0)
    assert W.wedge_3d(12).n == (95, 159, 95)                 # 64 x 128 x 64 cells


@pytest.mark.parametrize("k0,cells", W.IONIZATION_TABLE8)
def test_ionization_model(k0, cells):
    wl = W.ionization_2d(k0, cells)
    h = 50.0 / cells
    assert wl.h == (h, h)
    # Dirichlet on x = 0 and y = 0 (no layer; the first node is at h), ECS
    # beyond x = 50 and y = 50
    assert wl.ecs_lo == (0, 0) and wl.ecs_hi == (cells // 4,) * 2
    x = _coords(wl, 0)
    assert x[0] == h and x[cells - 1] == 50.0
    X, Y = np.meshgrid(x, x)
    np.testing.assert_allclose(wl.k2, np.exp(-X ** 2) + np.exp(-Y ** 2) + k0 ** 2, rtol=1e-15)
    np.testing.assert_allclose(wl.f[0].real, np.exp(-(X ** 2 + Y ** 2)), rtol=1e-15)
    assert not wl.f[0].imag.any()
    # the largest k sits next to the origin: sqrt(2 + k0^2) at most
    assert math.sqrt(wl.k2.max()) <= math.sqrt(2 + k0 * k0)
    # 5 2^q - 1 points per axis, down to 4 x 4
    assert H.auto_levels(wl.n) == int(math.log2(cells)) - 1
