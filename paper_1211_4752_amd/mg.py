"""ctypes binding of libmg.so (include/mg.h).

Argument marshalling only: every step of the method runs in the HIP library.
Grid vectors are torch complex128 tensors on the current HIP device, shaped
(nrhs, n_z, n_y, n_x) or (nrhs, n_y, n_x) (x fastest, as at the C ABI); k^2
and gradients are float64 tensors shaped like the grid.  Calls are ordered on
torch's current stream at construction time.
"""

from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmg.so")

MG_OK, MG_NOT_CONVERGED = 0, 1
MG_E_INVAL, MG_E_NOMEM, MG_E_DEVICE, MG_E_DIVERGED, MG_E_STATE = -1, -2, -3, -4, -5
PREC_C128, PREC_MIXED = 0, 1
MODE_STANDALONE, MODE_GMRES, MODE_FGMRES = 0, 1, 2
SMOOTH_JACOBI, SMOOTH_GMRES3 = 0, 1
MODES = {"standalone": MODE_STANDALONE, "gmres": MODE_GMRES, "fgmres": MODE_FGMRES}
KERNEL_CLASSES = [
    "smooth_restrict_fine", "prolong_smooth_fine", "coarse_levels", "coarsest_solve",
    "residual", "matvec_dot", "update_dot", "update_norm", "reduce", "combine", "other",
    "smooth_power_fine", "smooth_gram_fine", "smooth_gram_post_fine",
]

# every symbol include/mg.h declares
EXPORTS = [
    "mg_params_default", "mg_setup", "mg_cycle", "mg_solve", "mg_solve_adjoint",
    "mg_grad_k2", "mg_apply", "mg_num_levels", "mg_level_dims", "mg_get_sigma",
    "mg_profile", "mg_profile_read", "mg_destroy", "mg_status_str",
    "mg_tile_shape", "mg_batch_create", "mg_batch_solve", "mg_batch_destroy", "mg_cycle_noalloc",
]


class Params(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("h", ctypes.c_double * 3),
        ("nlevels", ctypes.c_int),
        ("ecs_lo", ctypes.c_int * 3),
        ("ecs_hi", ctypes.c_int * 3),
        ("ecs_angle", ctypes.c_double),
        ("sigma", ctypes.POINTER(ctypes.c_double)),
        ("theta_max", ctypes.c_double),
        ("nu1", ctypes.c_int),
        ("nu2", ctypes.c_int),
        ("omega", ctypes.c_double * 2),
        ("precision", ctypes.c_int),
        ("nrhs", ctypes.c_int),
        ("smoother", ctypes.c_int),
    ]


class MGError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__("%s: %s (%d)" % (what, lib().mg_status_str(status).decode(), status))


_lib = None


def lib():
    """Load libmg.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmg.so is not built (run python -m paper_1211_4752_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
        L.mg_params_default.argtypes = [ctypes.POINTER(Params)]
        L.mg_params_default.restype = None
        L.mg_setup.argtypes = [ctypes.POINTER(Params), vp, vp, ctypes.POINTER(vp)]
        L.mg_cycle.argtypes = [vp, vp, vp, dp]
        L.mg_cycle_noalloc.argtypes = [vp, vp, vp, dp]
        L.mg_solve.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, ip, dp]
        L.mg_solve_adjoint.argtypes = L.mg_solve.argtypes
        L.mg_grad_k2.argtypes = [vp, vp, vp, vp]
        L.mg_apply.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp]
        L.mg_num_levels.argtypes = [vp]
        L.mg_level_dims.argtypes = [vp, ctypes.c_int, ip]
        L.mg_get_sigma.argtypes = [vp, dp]
        L.mg_profile.argtypes = [vp, ctypes.c_int]
        L.mg_profile_read.argtypes = [vp, ctypes.c_int, dp, ctypes.POINTER(ctypes.c_longlong), dp]
        L.mg_destroy.argtypes = [vp]
        L.mg_destroy.restype = None
        L.mg_tile_shape.argtypes = [vp, ctypes.c_int, ctypes.c_int]
        L.mg_tile_shape.restype = ctypes.c_int
        L.mg_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(vp)]
        L.mg_batch_create.restype = ctypes.c_int
        L.mg_batch_solve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_int, ip, dp]
        L.mg_batch_solve.restype = ctypes.c_int
        L.mg_batch_destroy.argtypes = [vp]
        L.mg_batch_destroy.restype = None
        L.mg_status_str.argtypes = [ctypes.c_int]
        L.mg_status_str.restype = ctypes.c_char_p
        for name in ("mg_setup", "mg_cycle", "mg_cycle_noalloc", "mg_solve", "mg_solve_adjoint", "mg_grad_k2", "mg_apply",
                     "mg_level_dims", "mg_get_sigma", "mg_profile", "mg_profile_read"):
            getattr(L, name).restype = ctypes.c_int
        L.mg_num_levels.restype = ctypes.c_int
        _lib = L
    return _lib


def default_params() -> Params:
    p = Params()
    lib().mg_params_default(ctypes.byref(p))
    return p


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """Level hierarchy of one grid (mg_setup) and the calls on it.

    n: interior points per axis, x first; h: spacing per axis (scalar or
    per axis); k2: float64 device tensor shaped like the grid (slowest axis
    first); ecs: cells of the absorbing layer, an int for all sides or
    (lo, hi) tuples per axis; sigma: per-level complex shifts (None: default
    schedule with theta_max); precision: "c128" or "mixed"; smoother:
    "jacobi" (omega-Jacobi) or "gmres3" (one GMRES(3) cycle per smoothing
    step; GMRES mode then runs flexible GMRES).
    """

    def __init__(self, n, h, k2, *, ecs=0, ecs_angle=math.pi / 4, sigma=None,
                 theta_max=math.pi / 6, omega=2.0 / 3.0, precision="c128", nrhs=1,
                 nlevels=0, stream=None, smoother="jacobi"):
        import torch
        self.torch = torch
        self.n = tuple(int(v) for v in n)
        self.dim = len(self.n)
        p = default_params()
        p.ndim = self.dim
        hs = h if isinstance(h, (tuple, list)) else (h,) * self.dim
        for a in range(self.dim):
            p.n[a] = self.n[a]
            p.h[a] = float(hs[a])
        if isinstance(ecs, int):
            lo = hi = (ecs,) * self.dim
        else:
            lo, hi = ecs
        for a in range(self.dim):
            p.ecs_lo[a] = int(lo[a])
            p.ecs_hi[a] = int(hi[a])
        p.ecs_angle = float(ecs_angle)
        p.theta_max = float(theta_max)
        om = complex(omega)
        p.omega[0], p.omega[1] = om.real, om.imag
        p.precision = {"c128": PREC_C128, "mixed": PREC_MIXED}[precision]
        p.nrhs = int(nrhs)
        p.nlevels = int(nlevels)
        p.smoother = {"jacobi": SMOOTH_JACOBI, "gmres3": SMOOTH_GMRES3}[smoother]
        self.smoother = smoother
        self._sigma_buf = None
        if sigma is not None:
            s = np.asarray(sigma, dtype=np.complex128)
            self._sigma_buf = np.ascontiguousarray(np.stack([s.real, s.imag], axis=1).ravel())
            p.sigma = self._sigma_buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.params = p
        self.nrhs = int(nrhs)
        self.precision = precision
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.k2 = self._check_real(k2)
        ctx = ctypes.c_void_p()
        st = lib().mg_setup(ctypes.byref(p), _ptr(self.k2), ctypes.c_void_p(stream.cuda_stream),
                            ctypes.byref(ctx))
        if st != MG_OK:
            raise MGError(st, "mg_setup")
        self.ctx = ctx

    # -- checks -------------------------------------------------------------
    def _grid_shape(self, level=0):
        return tuple(reversed(self.level_dims(level)))

    def _check_real(self, t):
        torch = self.torch
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("expected a contiguous float64 device tensor")
        if tuple(t.shape) != tuple(reversed(self.n)):
            raise ValueError("expected shape %s, got %s" % (tuple(reversed(self.n)), tuple(t.shape)))
        return t

    def _check_vec(self, t, level=0):
        torch = self.torch
        if t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("expected a contiguous complex128 device tensor")
        shape = (self.nrhs,) + self._grid_shape(level)
        if tuple(t.shape) != shape:
            raise ValueError("expected shape %s, got %s" % (shape, tuple(t.shape)))
        return t

    def empty(self, level=0):
        return self.torch.zeros((self.nrhs,) + self._grid_shape(level), dtype=self.torch.complex128,
                                device=self.k2.device)

    # -- calls ----------------------------------------------------------------
    def level_dims(self, level):
        if not hasattr(self, "ctx"):
            return self.n
        out = (ctypes.c_int * 3)()
        st = lib().mg_level_dims(self.ctx, level, out)
        if st != MG_OK:
            raise MGError(st, "mg_level_dims")
        return tuple(out[a] for a in range(self.dim))

    @property
    def num_levels(self):
        return lib().mg_num_levels(self.ctx)

    def sigma(self):
        L = self.num_levels
        buf = (ctypes.c_double * (2 * L))()
        st = lib().mg_get_sigma(self.ctx, buf)
        if st != MG_OK:
            raise MGError(st, "mg_get_sigma")
        a = np.array(buf[:])
        return a[0::2] + 1j * a[1::2]

    def cycle(self, u, f, residual=False):
        self._check_vec(u)
        self._check_vec(f)
        res = (ctypes.c_double * self.nrhs)() if residual else None
        st = lib().mg_cycle(self.ctx, _ptr(u), _ptr(f), res)
        if st != MG_OK:
            raise MGError(st, "mg_cycle")
        return np.array(res[:]) if residual else None

    def cycle_noalloc(self, u, f, residual=False):
        """mg_cycle_noalloc: the cycle with the library's fixed scratch."""
        self._check_vec(u)
        self._check_vec(f)
        res = (ctypes.c_double * self.nrhs)() if residual else None
        st = lib().mg_cycle_noalloc(self.ctx, _ptr(u), _ptr(f), res)
        if st != MG_OK:
            raise MGError(st, "mg_cycle_noalloc")
        return np.array(res[:]) if residual else None

    def _solve(self, fn, u, f, mode, rtol, maxit, restart):
        self._check_vec(u)
        self._check_vec(f)
        its = (ctypes.c_int * self.nrhs)()
        hist = np.empty(self.nrhs * (maxit + 1), dtype=np.float64)
        mode_id = MODES[mode]
        st = fn(self.ctx, _ptr(u), _ptr(f), mode_id, float(rtol), int(maxit), int(restart), its,
                hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        if st not in (MG_OK, MG_NOT_CONVERGED, MG_E_DIVERGED):
            raise MGError(st, fn.__name__)
        hist = hist.reshape(self.nrhs, maxit + 1)
        hists = [h[h >= 0] for h in hist]
        status = {MG_OK: "converged", MG_NOT_CONVERGED: "not_converged", MG_E_DIVERGED: "diverged"}[st]
        return status, list(its[:]), hists

    def solve(self, u, f, mode="gmres", rtol=1e-6, maxit=1000, restart=20):
        """Solve in place on u; returns (status, iterations per rhs, histories)."""
        return self._solve(lib().mg_solve, u, f, mode, rtol, maxit, restart)

    def solve_adjoint(self, lam, g, mode="gmres", rtol=1e-6, maxit=1000, restart=20):
        return self._solve(lib().mg_solve_adjoint, lam, g, mode, rtol, maxit, restart)

    def grad_k2(self, u, lam, grad):
        self._check_vec(u)
        self._check_vec(lam)
        self._check_real(grad)
        st = lib().mg_grad_k2(self.ctx, _ptr(u), _ptr(lam), _ptr(grad))
        if st != MG_OK:
            raise MGError(st, "mg_grad_k2")
        return grad

    def apply(self, x, level=0, adjoint=False, out=None):
        self._check_vec(x, level)
        y = self.empty(level) if out is None else self._check_vec(out, level)
        st = lib().mg_apply(self.ctx, int(level), int(bool(adjoint)), _ptr(x), _ptr(y))
        if st != MG_OK:
            raise MGError(st, "mg_apply")
        return y

    def tile_shape(self, level, shape=-1):
        """Tile-shape id of the fused cycle kernels on a level; shape >= 0 sets it."""
        r = lib().mg_tile_shape(self.ctx, int(level), int(shape))
        if r < 0:
            raise MGError(r, "mg_tile_shape")
        return r

    def profile(self, enable=True):
        st = lib().mg_profile(self.ctx, int(bool(enable)))
        if st != MG_OK:
            raise MGError(st, "mg_profile")

    def profile_read(self):
        """{kernel class: (total ms, launches, algorithmic bytes)} since profile(True)."""
        out = {}
        for i, name in enumerate(KERNEL_CLASSES):
            ms = ctypes.c_double()
            cnt = ctypes.c_longlong()
            by = ctypes.c_double()
            st = lib().mg_profile_read(self.ctx, i, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(by))
            if st != MG_OK:
                raise MGError(st, "mg_profile_read")
            out[name] = (ms.value, cnt.value, by.value)
        return out

    def close(self):
        if getattr(self, "ctx", None):
            lib().mg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_STATUS = {MG_OK: "converged", MG_NOT_CONVERGED: "not_converged", MG_E_DIVERGED: "diverged"}


class Batch:
    """Several Solvers (grids of different sizes, same dimension, precision
    and stream) iterated together by mg_batch_solve: each kernel launch of a
    step covers the right-hand sides of all of them.  Borrows the solvers;
    close it before them."""

    def __init__(self, solvers):
        self.solvers = list(solvers)
        arr = (ctypes.c_void_p * len(self.solvers))(*[s.ctx.value for s in self.solvers])
        b = ctypes.c_void_p()
        st = lib().mg_batch_create(arr, len(self.solvers), ctypes.byref(b))
        if st != MG_OK:
            raise MGError(st, "mg_batch_create")
        self.handle = b

    def solve(self, us, fs, mode="gmres", rtol=1e-6, maxit=1000, restart=20):
        """Solve in place on each us[i]; returns (status, per-solver iteration
        lists, per-solver history lists)."""
        k = len(self.solvers)
        if len(us) != k or len(fs) != k:
            raise ValueError("one u and one f per solver")
        for s, u, f in zip(self.solvers, us, fs):
            s._check_vec(u)
            s._check_vec(f)
        up = (ctypes.c_void_p * k)(*[u.data_ptr() for u in us])
        fp = (ctypes.c_void_p * k)(*[f.data_ptr() for f in fs])
        tot = sum(s.nrhs for s in self.solvers)
        its = (ctypes.c_int * tot)()
        hist = np.empty(tot * (maxit + 1), dtype=np.float64)
        mode_id = MODES[mode]
        st = lib().mg_batch_solve(self.handle, up, fp, mode_id, float(rtol), int(maxit), int(restart), its,
                                  hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        if st not in _STATUS:
            raise MGError(st, "mg_batch_solve")
        hist = hist.reshape(tot, maxit + 1)
        iters, hists, r = [], [], 0
        for s in self.solvers:
            iters.append(list(its[r:r + s.nrhs]))
            hists.append([h[h >= 0] for h in hist[r:r + s.nrhs]])
            r += s.nrhs
        return _STATUS[st], iters, hists

    def close(self):
        if getattr(self, "handle", None):
            lib().mg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
