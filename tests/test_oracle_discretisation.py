"""Pins of oracle/helmholtz.py against facts the paper and the mathematics fix.

* Dirichlet eigenpairs of -Delta^h - sigma k^2 (Sec. 2.1: eigenvectors
  sin(l j pi / n), Laplacian eigenvalues (4/h^2) sin^2(l pi / 2n) per axis).
* Largest Laplacian eigenvalue 4d/h^2 (Sec. 2.1; the bound printed as
  2^{d+1}/h^2 coincides only for d <= 2).
* Second-order accuracy on a manufactured solution.
* ECS reading: uniform stencil at angle 0, complex symmetry of W A, and an
  outgoing discrete wave in 1D (Sec. 2.4).
* The printed per-level perturbations d-theta of Tables 1, 2 and 5 (Sec. 3.1,
  d-theta = theta_max / p).
"""

import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import helmholtz as H


def _grid_modes(n, modes):
    """Tensor sine mode on n^d interior points, array order slowest first."""
    j = np.arange(1, n + 1)
    N = n + 1
    vecs = [np.sin(m * j * math.pi / N) for m in modes]        # x first
    out = vecs[0]
    for v in vecs[1:]:
        out = np.multiply.outer(v, out)
    return out


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_dirichlet_eigenpairs(dim):
    n = 15 if dim < 3 else 7
    h = 1.0 / (n + 1)
    k = 9.0
    sigma = np.exp(0.3j)
    k2 = np.full((n,) * dim, k * k)
    A = H.operator(H.Problem((n,) * dim, (h,) * dim, k2), sigma)
    rng = np.random.default_rng(0)
    for _ in range(5):
        modes = rng.integers(1, n + 1, size=dim)
        w = _grid_modes(n, modes).ravel()
        lam = sum(4.0 / h ** 2 * math.sin(m * math.pi / (2 * (n + 1))) ** 2
                  for m in modes) - sigma * k * k
        np.testing.assert_allclose(A @ w, lam * w, rtol=0, atol=1e-11 * abs(lam) * np.abs(w).max() + 1e-9)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_laplacian_spectrum_bound(dim):
    n = 15 if dim < 3 else 7
    h = 1.0 / (n + 1)
    A = H.operator(H.Problem((n,) * dim, (h,) * dim, np.zeros((n,) * dim)))
    ev = np.linalg.eigvalsh(A.toarray().real)
    assert ev.min() > 0
    assert ev.max() < 4 * dim / h ** 2
    # the top mode approaches the bound: 4d/h^2 sin^2(n pi / 2(n+1))
    top = 4 * dim / h ** 2 * math.sin(n * math.pi / (2 * (n + 1))) ** 2
    assert ev.max() == pytest.approx(top, rel=1e-12)


def test_manufactured_solution_second_order():
    k = 5.0          # k^2 = 25 lies between the eigenvalues 2 pi^2 and 5 pi^2
    errs = []
    for n in (15, 31, 63, 127):
        h = 1.0 / (n + 1)
        x = h * np.arange(1, n + 1)
        X, Y = np.meshgrid(x, x, indexing="xy")      # array [y, x]
        u_star = np.sin(math.pi * X) * np.sin(2 * math.pi * Y)
        f = (5 * math.pi ** 2 - k * k) * u_star
        A = H.operator(H.Problem((n, n), (h, h), np.full((n, n), k * k)))
        u = spla.spsolve(A.tocsc(), f.ravel().astype(complex))
        errs.append(np.abs(u - u_star.ravel()).max())
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.8 < r < 4.2 for r in ratios), ratios


def test_ecs_zero_angle_is_uniform():
    n, h = 31, 1.0 / 32
    z = H.ecs_nodes(n, h, 1.0, 8 * h, 8 * h, 0.0)
    cm, c0, cp = H.axis_coefficients(z)
    np.testing.assert_allclose(cm, -1 / h ** 2, rtol=1e-13)
    np.testing.assert_allclose(cp, -1 / h ** 2, rtol=1e-13)
    np.testing.assert_allclose(c0, 2 / h ** 2, rtol=1e-13)


def test_ecs_layer_geometry():
    n, h = 31, 1.0 / 32
    phi = math.pi / 4
    z = H.ecs_nodes(n, h, 1.0, 8 * h, 4 * h, phi)
    x = h * np.arange(n + 2)
    inside = (x >= 8 * h) & (x <= 1 - 4 * h)
    np.testing.assert_array_equal(z[inside], x[inside])
    # outside the physical region the spacing is h rotated by e^{i phi}
    # (pointing outward), so |Im z| grows towards both edges
    assert z[0] == pytest.approx(8 * h - 8 * h * np.exp(1j * phi))
    assert z[-1] == pytest.approx(1 - 4 * h + 4 * h * np.exp(1j * phi))
    assert np.all(np.diff(np.abs(z[:9].imag)) < 0)
    assert np.all(np.diff(np.abs(z[-5:].imag)) > 0)


def test_ecs_complex_symmetry():
    """W A is complex symmetric with W = (x)_axes diag((hm + hp) / 2)."""
    n = 15
    h = 1.0 / 16
    rng = np.random.default_rng(1)
    k2 = 100 + 20 * rng.random((n, n))
    lev = H.build_hierarchy(H.Problem((n, n), (h, h), k2, (4, 3), (2, 5), math.pi / 5),
                            nlevels=1)[0]
    W = np.multiply.outer(lev.weights[1], lev.weights[0]).ravel()
    WA = (W[:, None] * lev.A.toarray())
    np.testing.assert_allclose(WA, WA.T, rtol=0, atol=1e-12 * np.abs(WA).max())
    assert np.abs(lev.A.toarray() - lev.A.toarray().T).max() > 1e-3 * np.abs(WA).max() / np.abs(W).max()


@pytest.mark.parametrize("kh", [0.5, 0.25])
def test_ecs_outgoing_wave_1d(kh):
    """In the physical region the 1D solution is the discrete outgoing Green's
    function C e^{i kappa h |j - j0|}, cos(kappa h) = 1 - (kh)^2 / 2,
    C = i h^2 / (2 sin(kappa h)), up to an O((kh)^2) reflection at the layer."""
    n, ecs = 255, 32
    h = 1.0 / (n + 1)
    k = kh / h
    A = H.operator(H.Problem((n,), (h,), np.full(n, k * k), (ecs,), (ecs,), math.pi / 4))
    j0 = (n - 1) // 2
    f = np.zeros(n, complex)
    f[j0] = 1.0
    u = spla.spsolve(A.tocsc(), f)
    kap_h = math.acos(1 - kh * kh / 2)
    C = 1j * h * h / (2 * math.sin(kap_h))
    j = np.arange(n)
    phys = (j >= ecs) & (j < n - ecs)
    g = C * np.exp(1j * kap_h * np.abs(j - j0))
    err = np.abs(u[phys] - g[phys]).max() / abs(C)
    assert err < 0.2 * kh * kh
    # inside the layer the outgoing wave decays like exp(-k Im z); a wrongly
    # rotated (incoming) layer would grow instead
    decay = math.exp(-kh * (ecs - 2) * math.sin(math.pi / 4))
    assert abs(u[2]) < 2 * decay * abs(u[j0])


@pytest.mark.parametrize("kh", [0.5, 0.25])
def test_ecs_one_sided_outgoing_wave_1d(kh):
    """Dirichlet wall at x = 0 (no layer there), ECS layer at the far end:
    by the image method the discrete solution in the physical region is
    C (e^{i kappa h |m - m0|} - e^{i kappa h (m + m0)}), m the node number
    counted from the wall, which vanishes at the wall and is outgoing beyond
    the source."""
    n, ecs = 255, 32
    h = 1.0 / (n + 1)
    k = kh / h
    A = H.operator(H.Problem((n,), (h,), np.full(n, k * k), (0,), (ecs,), math.pi / 4))
    j0 = 60
    f = np.zeros(n, complex)
    f[j0] = 1.0
    u = spla.spsolve(A.tocsc(), f)
    kap_h = math.acos(1 - kh * kh / 2)
    C = 1j * h * h / (2 * math.sin(kap_h))
    m, m0 = np.arange(n) + 1, j0 + 1
    g = C * (np.exp(1j * kap_h * np.abs(m - m0)) - np.exp(1j * kap_h * (m + m0)))
    phys = m < n + 1 - ecs
    # the layer's O((kh)^2) reflection, relative to the amplitude 2 |C| of
    # the two-wave solution
    err = np.abs(u[phys] - g[phys]).max() / (2 * abs(C))
    assert err < 0.2 * kh * kh
    # the same problem with a wrong (mirror-free) Green's function is far off
    g_free = C * np.exp(1j * kap_h * np.abs(m - m0))
    assert np.abs(u[phys] - g_free[phys]).max() / abs(C) > 0.5


def test_anisotropic_rectangular_eigenpairs():
    """Per-axis sizes and spacings (the wedge and ionization grids): on
    n_x x n_y points with spacings h_x != h_y, tensor sine modes are
    eigenvectors with eigenvalue sum_a (4/h_a^2) sin^2(l_a pi / 2(n_a+1))
    - sigma k^2."""
    n, h = (11, 23), (0.3, 0.17)
    k2, sigma = 40.0, np.exp(0.2j)
    A = H.operator(H.Problem(n, h, np.full((n[1], n[0]), k2)), sigma)
    for lx, ly in [(1, 1), (3, 17), (11, 2), (6, 23)]:
        wx = np.sin(lx * np.arange(1, n[0] + 1) * math.pi / (n[0] + 1))
        wy = np.sin(ly * np.arange(1, n[1] + 1) * math.pi / (n[1] + 1))
        w = np.multiply.outer(wy, wx).ravel()
        lam = (4 / h[0] ** 2 * math.sin(lx * math.pi / (2 * (n[0] + 1))) ** 2
               + 4 / h[1] ** 2 * math.sin(ly * math.pi / (2 * (n[1] + 1))) ** 2 - sigma * k2)
        np.testing.assert_allclose(A @ w, lam * w, rtol=0, atol=1e-12 * abs(lam) + 1e-10)


def test_printed_dtheta_values():
    """Tables 1, 2 and 5 print d-theta = theta_max / p, p the number of levels
    of an n = 2^p interval grid coarsened down to one point."""
    table1 = {32: 30, 64: 36, 128: 42, 256: 48, 512: 54, 1024: 60}
    table2 = {64: 36, 128: 42, 256: 48, 512: 54, 1024: 60, 2048: 66}
    for tab in (table1, table2):
        for n, denom in tab.items():
            p = int(round(math.log2(n)))
            th = H.theta_schedule(p, math.pi / 6)
            assert th[1] == pytest.approx(math.pi / denom, rel=1e-14)
    table5 = {15: 105, 12: 84, 10: 70, 8: 56, 6: 42, 5: 35, 4: 28}
    for tmax, denom in table5.items():
        th = H.theta_schedule(7, math.pi / tmax)        # n = 128, p = 7
        assert th[1] == pytest.approx(math.pi / denom, rel=1e-14)
    # a 2^p - 1 interior grid coarsened to one point has p levels
    n = 2 ** 5 - 1
    levels = H.build_hierarchy(H.Problem((n,), (1 / 32,), np.zeros(n)), nlevels=5)
    assert [lv.n[0] for lv in levels] == [31, 15, 7, 3, 1]


def test_schedule_endpoints():
    s = H.sigma_schedule(9, math.pi / 6)
    assert s[0] == 1.0
    np.testing.assert_allclose(np.angle(s), np.arange(9) * math.pi / 54, atol=1e-15)
    b = H.sigma_schedule(9, math.pi / 6, kind="beta")
    np.testing.assert_allclose(b.imag, np.tan(np.arange(9) * math.pi / 54), rtol=1e-14)
    np.testing.assert_allclose(b.real, 1.0)


def test_hierarchy_sizes_and_injection():
    assert H.auto_levels((63, 63)) == 5
    assert H.auto_levels((1023, 1023)) == 9
    assert H.auto_levels((255, 255, 255)) == 7
    assert H.auto_levels((159, 159)) == 6        # 159 79 39 19 9 4
    assert H.auto_levels((223, 223)) == 6        # ... 13 6
    k2 = np.arange(15 * 15, dtype=float).reshape(15, 15)
    c = H.inject_k2(k2)
    assert c.shape == (7, 7)
    assert c[2, 3] == k2[5, 7]
