"""Pins of oracle/cycle.py against the paper's two-grid analysis and brute force.

* Sine-mode identities of full weighting and linear interpolation (Sec. 2.1):
  R w_l = c_l w_l^{2h}, R w_{l'} = -s_l w_l^{2h}, P w_l^{2h} = c_l w_l - s_l w_{l'}.
* Two-grid operator on sine modes (Sec. 2.1, eq. tgsmoo and its companion for
  w_{l'}, whose sign is printed as '-' but must be '+' for w_{l'} =
  sin((n-l) j pi / n); both forms are checked against the oracle's cycle and
  the printed sign is shown to fail), 1D and the 2D tensor form, with the
  level-dependent shifts of eq. cslvariant.
* Smooth-mode factor (Sec. 3.1.1, eq. cslexp): TG^m w_l ~ (1 - e^{-i dtheta}) w_l.
* Perturbation spectrum gamma (Sec. 3.1.2, eq. gamk), zero for k = 0
  (eq. eigzero, the Poisson invariant).
* The full multilevel cycle against explicitly formed error-propagation
  matrices on tiny grids (brute force, independent formulation).
* Standalone convergence on a definite problem to the sparse direct solution.
"""

import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import cycle as C
from oracle import helmholtz as H


def _cs(l, n):
    return math.cos(l * math.pi / (2 * n)) ** 2, math.sin(l * math.pi / (2 * n)) ** 2


def test_transfer_sine_identities_1d():
    n = 32                                   # intervals; n - 1 interior points
    j = np.arange(1, n)
    J = np.arange(1, n // 2)
    R = C.restriction_1d(n - 1).toarray()
    P = C.prolongation((n - 1,)).toarray()
    for l in range(1, n // 2):
        c, s = _cs(l, n)
        w = np.sin(l * j * math.pi / n)
        wp = np.sin((n - l) * j * math.pi / n)
        wc = np.sin(l * J * math.pi / (n // 2))
        np.testing.assert_allclose(R @ w, c * wc, atol=1e-14)
        np.testing.assert_allclose(R @ wp, -s * wc, atol=1e-14)
        np.testing.assert_allclose(P @ wc, c * w - s * wp, atol=1e-14)


def test_transfer_2d_tensor():
    n = 16
    j = np.arange(1, n)
    J = np.arange(1, n // 2)
    R = C.restriction((n - 1, n - 1))
    P = C.prolongation((n - 1, n - 1))
    l, m = 3, 5
    cl, sl = _cs(l, n)
    cm, sm = _cs(m, n)
    wl, wlp = np.sin(l * j * math.pi / n), np.sin((n - l) * j * math.pi / n)
    wm, wmp = np.sin(m * j * math.pi / n), np.sin((n - m) * j * math.pi / n)
    wc = np.multiply.outer(np.sin(m * J * math.pi / 8), np.sin(l * J * math.pi / 8)).ravel()
    w = np.multiply.outer(wm, wl).ravel()         # [y, x]: x mode l, y mode m
    np.testing.assert_allclose(R @ w, cl * cm * wc, atol=1e-14)
    np.testing.assert_allclose(P @ wc, np.multiply.outer(cm * wm - sm * wmp, cl * wl - sl * wlp).ravel(),
                               atol=1e-14)


def _two_grid(n, k, sig, nu=0, dim=1):
    N = n - 1
    h = 1.0 / n
    prob = H.Problem((N,) * dim, (h,) * dim, np.full((N,) * dim, k * k))
    levels = H.build_hierarchy(prob, sigma=np.array(sig), nlevels=2)
    return levels, C.VCycle(levels, nu1=nu, nu2=nu)


def _tg_apply(levels, vc, e):
    """Error after one correction without smoothing: e - M A~_0 e."""
    f = levels[0].A @ e
    return e - vc(np.zeros_like(f), f)


def test_two_grid_closed_form_1d():
    n, k = 32, 25.0
    h = 1.0 / n
    sig = [np.exp(0.05j), np.exp(0.15j)]        # fine theta_{m-1}, coarse theta_m
    levels, vc = _two_grid(n, k, sig)
    j = np.arange(1, n)
    printed_sign_fails = []
    for l in range(1, n // 2):
        c, s = _cs(l, n)
        w = np.sin(l * j * math.pi / n)
        wp = np.sin((n - l) * j * math.pi / n)
        lam_h = 4 / h ** 2 * s - sig[0] * k * k
        lam_hp = 4 / h ** 2 * c - sig[0] * k * k
        lam_H = 4 / h ** 2 * s * c - sig[1] * k * k
        mix = c * w - s * wp
        np.testing.assert_allclose(_tg_apply(levels, vc, w), w - c * lam_h / lam_H * mix, atol=1e-12)
        got = _tg_apply(levels, vc, wp)
        np.testing.assert_allclose(got, wp + s * lam_hp / lam_H * mix, atol=1e-12)
        printed_sign_fails.append(np.abs(got - (wp - s * lam_hp / lam_H * mix)).max() > 1e-3)
    assert all(printed_sign_fails)


def test_two_grid_closed_form_2d_tensor():
    n, k = 16, 12.0
    h = 1.0 / n
    sig = [1.0, np.exp(0.2j)]
    levels, vc = _two_grid(n, k, sig, dim=2)
    j = np.arange(1, n)
    for l, m in [(1, 1), (2, 5), (7, 3)]:
        cl, sl = _cs(l, n)
        cm, sm = _cs(m, n)
        w = np.multiply.outer(np.sin(m * j * math.pi / n), np.sin(l * j * math.pi / n)).ravel()
        mix = np.multiply.outer(cm * np.sin(m * j * math.pi / n) - sm * np.sin((n - m) * j * math.pi / n),
                                cl * np.sin(l * j * math.pi / n) - sl * np.sin((n - l) * j * math.pi / n)).ravel()
        lam_h = 4 / h ** 2 * (sl + sm) - sig[0] * k * k
        lam_H = 4 / h ** 2 * (sl * cl + sm * cm) - sig[1] * k * k
        np.testing.assert_allclose(_tg_apply(levels, vc, w), w - cl * cm * lam_h / lam_H * mix, atol=1e-12)


def test_smooth_mode_factor():
    """For l << n/2 with lambda_L << k^2 the w_l coefficient of TG^m w_l is
    about 1 - e^{-i dtheta}; smooth modes are not amplified (|.| < 1)."""
    n, k = 256, 100.0
    dth = math.pi / 48
    levels, vc = _two_grid(n, k, [1.0, np.exp(1j * dth)])
    j = np.arange(1, n)
    w = np.sin(j * math.pi / n)
    t = _tg_apply(levels, vc, w)
    coef = np.vdot(w, t) / np.vdot(w, w)
    assert abs(coef - (1 - np.exp(-1j * dth))) < 2e-3
    assert abs(coef) < 1
    # standard (unshifted) coarse grid maps the smooth mode to ~0
    levels0, vc0 = _two_grid(n, k, [1.0, 1.0])
    coef0 = np.vdot(w, _tg_apply(levels0, vc0, w)) / np.vdot(w, w)
    assert abs(coef0) < 1e-2 * abs(coef)
    # |1 - e^{-i dtheta}| < 1 exactly when dtheta < pi/3 (Sec. 3.1.1)
    for d in np.linspace(0.01, math.pi, 50):
        assert (abs(1 - np.exp(-1j * d)) < 1) == (d < math.pi / 3)


@pytest.mark.parametrize("k", [0.0, 30.0])
def test_gamma_spectrum(k):
    """Eigenvalues of A~_c^{-1}(A_c - A~_c) on the coarse grid equal
    k^2 (e^{i dtheta} - 1) / (lambda_L - k^2 e^{i dtheta}) (eq. gamk)."""
    n = 32
    N = (n // 2) - 1
    H2 = 2.0 / n
    dth = 0.2
    k2 = np.full(N, k * k)
    A_c = H.operator(H.Problem((N,), (H2,), k2), 1.0).toarray()
    At_c = H.operator(H.Problem((N,), (H2,), k2), np.exp(1j * dth)).toarray()
    got = np.linalg.eigvals(np.linalg.solve(At_c, A_c - At_c))
    J = np.arange(1, N + 1)
    lamL = 4 / H2 ** 2 * np.sin(J * math.pi / (2 * (N + 1))) ** 2
    want = k * k * (np.exp(1j * dth) - 1) / (lamL - k * k * np.exp(1j * dth))
    got = got[np.argsort(got.real + 1e3 * got.imag)]
    want = want[np.argsort(want.real + 1e3 * want.imag)]
    np.testing.assert_allclose(got, want, atol=1e-12)
    if k == 0:
        assert np.abs(got).max() < 1e-14


def test_poisson_invariant():
    """k = 0: the level-dependent cycle equals the standard cycle (eq. eigzero)."""
    n = 31
    prob = H.Problem((n, n), (1 / 32, 1 / 32), np.zeros((n, n)), (4, 4), (4, 4))
    rng = np.random.default_rng(3)
    u0 = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    f = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    a = C.VCycle(H.build_hierarchy(prob))(u0, f)
    b = C.VCycle(H.build_hierarchy(prob, sigma=np.ones(4)))(u0, f)
    np.testing.assert_array_equal(a, b)


def _brute_force_affine(levels, nu1, nu2, omega):
    """Error propagation E_l and cycle map M_l from dense matrices:
    S = I - omega D^{-1} A~, M_{L-1} = A~^{-1},
    E_l = S^{nu2} (I - P M_{l+1} R A~_l) S^{nu1}, M_l = (I - E_l) A~_l^{-1}."""
    L = len(levels)
    A = [lv.A.toarray() for lv in levels]
    M = [None] * L
    M[L - 1] = np.linalg.inv(A[L - 1])
    E0 = None
    for l in reversed(range(L - 1)):
        nl = A[l].shape[0]
        I = np.eye(nl)
        S = I - omega * A[l] / np.diag(A[l])[:, None]
        R = C.restriction(levels[l].n).toarray()
        P = 2.0 ** len(levels[l].n) * R.T
        E = np.linalg.matrix_power(S, nu2) @ (I - P @ M[l + 1] @ R @ A[l]) @ np.linalg.matrix_power(S, nu1)
        M[l] = (I - E) @ np.linalg.inv(A[l])
        if l == 0:
            E0 = E
    return E0, M[0]


@pytest.mark.parametrize("dim,n,nu", [(2, 15, (1, 1)), (2, 15, (2, 1)), (3, 7, (1, 1))])
def test_cycle_against_brute_force(dim, n, nu):
    h = 1.0 / (n + 1)
    rng = np.random.default_rng(11)
    k2 = (0.5 / h) ** 2 * (1 + 0.3 * rng.random((n,) * dim))
    ecs = (2,) * dim
    prob = H.Problem((n,) * dim, (h,) * dim, k2, ecs, ecs, math.pi / 4)
    levels = H.build_hierarchy(prob)
    assert len(levels) >= 2
    omega = 2.0 / 3.0
    vc = C.VCycle(levels, nu1=nu[0], nu2=nu[1], omega=omega)
    N = levels[0].size
    u0 = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    E, M = _brute_force_affine(levels, nu[0], nu[1], omega)
    want = E @ u0 + M @ f
    got = vc(u0, f)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-10 * np.abs(want).max())


def test_standalone_converges_on_definite_problem():
    """Poisson-like definite problem: the cycle converges to the direct solution."""
    n = 63
    h = 1.0 / 64
    prob = H.Problem((n, n), (h, h), np.full((n, n), 10.0))
    levels = H.build_hierarchy(prob)
    vc = C.VCycle(levels)
    f = np.zeros(n * n, complex)
    f[(n * n) // 2] = 1.0
    u, hist, its, status = C.standalone(vc, f, rtol=1e-10, maxit=60)
    assert status == "converged"
    assert its < 30
    # a V(1,1) damped-Jacobi cycle contracts by a grid-independent factor
    rate = (hist[its] / hist[0]) ** (1.0 / its)
    assert rate < 0.45
    exact = spla.spsolve(levels[0].A.tocsc(), f)
    assert np.linalg.norm(u - exact) / np.linalg.norm(exact) < 1e-8


def test_standalone_history_convention():
    n = 31
    prob = H.Problem((n, n), (1 / 32, 1 / 32), np.full((n, n), 10.0))
    vc = C.VCycle(H.build_hierarchy(prob))
    f = np.ones(n * n, complex)
    u, hist, its, status = C.standalone(vc, f, rtol=1e-6, maxit=50)
    assert hist[0] == pytest.approx(1.0)
    assert len(hist) == its + 1 and hist[its] <= 1e-6 < hist[its - 1]
    A = vc.A[0]
    # the returned iterate is one cycle past the first one within tolerance
    assert np.linalg.norm(f - A @ u) / np.linalg.norm(f) < hist[its]
