"""The C ABI library loads on a machine without a GPU and exports every entry
point that include/mg.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2601_02975_amd", "libmgcut.so")


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "mg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for want in ("mg_setup", "mg_solve", "mg_destroy", "mg_query", "mg_error_string", "mg_vcycle", "mg_rhs"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmgcut.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmgcut.so not built")
def test_host_only_calls():
    lib = ctypes.CDLL(LIB)
    lib.mg_error_string.restype = ctypes.c_char_p
    assert lib.mg_error_string(0) == b"ok"
    assert b"geometry" in lib.mg_error_string(-2)
    assert lib.mg_destroy(None) == 0
    # invalid arguments are rejected before any device work
    assert lib.mg_setup(None, 0, None, ctypes.c_double(1.0), ctypes.c_double(0.0), ctypes.c_double(1.0),
                        None, None, None) == -1


def _setup_args(mg, a=1.0, b=0.0, c=1.0, **opt):
    """An mg_setup call on the unit square (64^2) with the given coefficients
    and options, through the binding's structures (host-side checks only)."""
    import workloads as W
    carr, keep = mg._curves([W.box_curve(0.0, 0.0, 1.0, 1.0)])
    g = mg.mg_grid(0.0, 0.0, 1.0 / 64, 64, 64)
    o = mg._options(0.08, 0.5, (3, 3), 0, 16, mg.FP64, 100, 0)
    for k, v in opt.items():
        setattr(o, k, v)
    h = ctypes.c_void_p()
    code = mg.lib().mg_setup(ctypes.byref(g), 1, carr, a, b, c, ctypes.byref(o), None, ctypes.byref(h))
    assert not h.value
    return code


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmgcut.so not built")
@pytest.mark.parametrize("abc", [(1.0, 2.0, 1.0), (1.0, 3.0, 2.0), (-1.0, 0.0, 1.0), (0.0, 0.0, 1.0)])
def test_setup_rejects_a_non_elliptic_equation(abc):
    """b^2 - 4ac < 0 is required (eq. (1.1)); anything else is rejected
    before any device work."""
    import paper_2601_02975_amd as mg
    assert _setup_args(mg, *abc) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmgcut.so not built")
@pytest.mark.parametrize("opt,code", [({"degree": 3}, -8), ({"w_min": 0.0}, -1), ({"colouring": 2}, -1),
                                      ({"omega": 0.0}, -1), ({"small_cells": -2}, -1), ({"nu1": -1}, -1),
                                      ({"pair_sweeps": 1}, -1)])
def test_setup_rejects_bad_options(opt, code):
    import paper_2601_02975_amd as mg
    assert _setup_args(mg, **opt) == code


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmgcut.so not built")
def test_setup_rejects_nan_geometry():
    import paper_2601_02975_amd as mg
    import workloads as W
    carr, keep = mg._curves([W.box_curve(0.0, 0.0, 1.0, 1.0)])
    keep[0][1].p[2] = float("nan")
    g = mg.mg_grid(0.0, 0.0, 1.0 / 64, 64, 64)
    h = ctypes.c_void_p()
    assert mg.lib().mg_setup(ctypes.byref(g), 1, carr, 1.0, 0.0, 1.0, None, None, ctypes.byref(h)) == -1
