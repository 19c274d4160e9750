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
