"""The C-ABI library loads, exports every symbol include/mg.h declares, and
rejects invalid set-ups on the host before touching a device (no GPU needed)."""

import ctypes
import math
import os
import re

import pytest

from paper_1211_4752_amd import mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mg.h")

pytestmark = pytest.mark.skipif(not os.path.exists(mg.LIB_PATH), reason="libmg.so not built")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(mg.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(mg.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_params_default():
    p = mg.default_params()
    assert p.ndim == 2 and p.nu1 == 1 and p.nu2 == 1 and p.nrhs == 1
    assert p.omega[0] == pytest.approx(2 / 3) and p.omega[1] == 0
    assert p.theta_max == pytest.approx(math.pi / 6)
    assert p.ecs_angle == pytest.approx(math.pi / 4)
    assert p.precision == mg.PREC_C128 and p.nlevels == 0 and not p.sigma


def _setup(p, k2=8):
    ctx = ctypes.c_void_p()
    st = mg.lib().mg_setup(ctypes.byref(p), ctypes.c_void_p(k2), None, ctypes.byref(ctx))
    return st, ctx


def _params(n=(63, 63), **kw):
    p = mg.default_params()
    p.ndim = len(n)
    for a, m in enumerate(n):
        p.n[a] = m
        p.h[a] = 1.0 / (m + 1)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("bad", [
    dict(ndim=4), dict(ndim=1), dict(nrhs=0), dict(nu1=2), dict(nu2=0), dict(precision=7),
    dict(nlevels=-1),
])
def test_setup_rejects_invalid_params(bad):
    st, ctx = _setup(_params(**bad))
    assert st == mg.MG_E_INVAL and not ctx.value


def test_setup_rejects_bad_dimensions():
    assert _setup(_params((64, 64)))[0] == mg.MG_E_INVAL          # cannot coarsen at all
    assert _setup(_params((63, 64)))[0] == mg.MG_E_INVAL
    assert _setup(_params((63, 63), nlevels=7))[0] == mg.MG_E_INVAL  # 63 31 15 7 3 1 -> even step
    p = _params((127, 127), nlevels=2)                             # coarsest 63^2 > 1024 unknowns
    assert _setup(p)[0] == mg.MG_E_INVAL
    p = _params((63, 63))
    p.ecs_lo[0] = 40
    p.ecs_hi[0] = 40
    assert _setup(p)[0] == mg.MG_E_INVAL
    assert _setup(_params(), k2=0)[0] == mg.MG_E_INVAL


def test_null_handles():
    L = mg.lib()
    L.mg_destroy(None)
    assert L.mg_num_levels(None) == 0
    assert L.mg_cycle(None, None, None, None) == mg.MG_E_INVAL
    assert L.mg_solve(None, None, None, 1, 1e-6, 10, 20, None, None) == mg.MG_E_INVAL
    assert L.mg_apply(None, 0, 0, None, None) == mg.MG_E_INVAL
    out = ctypes.c_void_p(123)
    assert L.mg_setup(None, None, None, ctypes.byref(out)) == mg.MG_E_INVAL and not out.value
    assert L.mg_tile_shape(None, 0, -1) == mg.MG_E_INVAL
    assert L.mg_profile_read(None, 0, None, None, None) == mg.MG_E_INVAL


def test_batch_null_handles():
    L = mg.lib()
    L.mg_batch_destroy(None)
    out = ctypes.c_void_p(123)
    assert L.mg_batch_create(None, 1, ctypes.byref(out)) == mg.MG_E_INVAL and not out.value
    arr = (ctypes.c_void_p * 2)(None, None)
    out = ctypes.c_void_p(123)
    assert L.mg_batch_create(arr, 2, ctypes.byref(out)) == mg.MG_E_INVAL and not out.value
    assert L.mg_batch_create(arr, 0, ctypes.byref(out)) == mg.MG_E_INVAL
    assert L.mg_batch_create(arr, 1, None) == mg.MG_E_INVAL
    assert L.mg_batch_solve(None, None, None, 1, 1e-6, 10, 20, None, None) == mg.MG_E_INVAL


def test_status_strings():
    L = mg.lib()
    for code in (0, 1, -1, -2, -3, -4, -5):
        assert L.mg_status_str(code)
    assert L.mg_status_str(99) == b"unknown status"
