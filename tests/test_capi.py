"""C-ABI checks that need no GPU: the library builds and loads, exports every
entry point include/sgw.h declares, and rejects invalid problem descriptions
before touching the device."""

import ctypes
import os
import re

import pytest

import paper_2512_23027_amd as sgw
from paper_2512_23027_amd import build as sgw_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(sgw.LIBPATH):
        sgw_build.build()
    return sgw.lib()


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "sgw.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sgw_[a-z_]+)\s*\(", src)))


def test_header_declares_binding_exports():
    assert declared_symbols() == sorted(sgw.EXPORTS)


def test_library_exports_every_declared_symbol(L):
    for name in declared_symbols():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


def _desc(n=8, xs=(0, 4, 8), ys=(0, 4, 8)):
    d = sgw.ProblemDesc()
    d.n = n
    d.nsx, d.nsy = len(xs) - 1, len(ys) - 1
    xa = (ctypes.c_int * len(xs))(*xs)
    ya = (ctypes.c_int * len(ys))(*ys)
    d.xsplits = ctypes.cast(xa, ctypes.POINTER(ctypes.c_int))
    d.ysplits = ctypes.cast(ya, ctypes.POINTER(ctypes.c_int))
    d.L, d.p_in, d.p_out = 2, 2, 2
    d.sigma, d.bx, d.by = 0.2, 0.5, 0.5
    d.dt = 0.01
    return d, (xa, ya)


@pytest.mark.parametrize("mutate,expect", [
    (lambda d: setattr(d, "n", 1), "invalid problem description"),
    (lambda d: setattr(d, "dt", 0.0), "invalid problem description"),
    (lambda d: setattr(d, "bx", -1.0), "invalid problem description"),
])
def test_create_rejects_invalid_description(L, mutate, expect):
    d, keep = _desc()
    mutate(d)
    ctx = ctypes.c_void_p()
    rc = L.sgw_create(ctypes.byref(d), None, ctypes.byref(ctx))
    assert rc == -1
    assert expect in L.sgw_last_error(ctx).decode()
    L.sgw_destroy(ctx)


def test_create_rejects_bad_splits(L):
    for xs, ys, msg in [((0, 5, 9), (0, 4, 8), "start at 0 and end at n"),
                        ((0, 1, 8), (0, 4, 8), "at least 2 cells"),
                        ((0, 8), (0, 8), "at least two subdomains")]:
        d, keep = _desc(8, xs, ys)
        ctx = ctypes.c_void_p()
        rc = L.sgw_create(ctypes.byref(d), None, ctypes.byref(ctx))
        assert rc == -1, (xs, ys)
        assert msg in L.sgw_last_error(ctx).decode()
        L.sgw_destroy(ctx)


def test_null_arguments(L):
    assert L.sgw_create(None, None, None) == -1
    assert L.sgw_step(None, 1, None, None) == -1
    assert L.sgw_query(None, 0) == -1
    assert L.sgw_set_cheb_tile(None, 0, 0, 1, 0) == -1


@pytest.mark.parametrize("field,value", [("inner_prec", 7), ("cheb_degree", 65),
                                         ("precision", 3)])
def test_create_rejects_bad_solver_options(L, field, value):
    d, keep = _desc()
    setattr(d, field, value)
    ctx = ctypes.c_void_p()
    rc = L.sgw_create(ctypes.byref(d), None, ctypes.byref(ctx))
    assert rc == -1
    assert "out of range" in L.sgw_last_error(ctx).decode()
    L.sgw_destroy(ctx)
