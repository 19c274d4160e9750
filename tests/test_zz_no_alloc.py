"""mg_residual_norm_noalloc, the entry point for callers that cannot
allocate: its residual and norm against mg_residual's on the same handle,
through the C ABI, on two calls in a row (the second on a smaller level, so
that the fixed scratch still holds the first call's partial maxima)."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("name", ["three_disks128", "star128"])
def test_noalloc_residual_norm_matches_mg_residual(name):
    torch = _torch()
    import paper_2601_02975_amd as mg
    P = {"three_disks128": lambda: W.three_disks_config(0, 128), "star128": lambda: W.star_config(0, 128)}[name]()
    S = mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps)
    lib = mg.lib()
    lib.mg_residual_norm_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.mg_residual_norm_noalloc.restype = ctypes.c_int
    rng = np.random.default_rng(41)
    for level in (0, 1):                          # the second call is on the smaller level
        ny, nx = S.padded_shape(level)
        u = torch.tensor(rng.standard_normal((ny, nx)), device="cuda")
        b = torch.tensor(rng.standard_normal((ny, nx)), device="cuda")
        r_ref = torch.zeros_like(u)
        n_ref = S.residual(level, b, u, r_ref)
        r_na = torch.full_like(u, 7.0)
        n_na = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        code = lib.mg_residual_norm_noalloc(S.h, level, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                            ctypes.c_void_p(r_na.data_ptr()), ctypes.c_void_p(n_na.data_ptr()),
                                            mg._stream())
        assert code == 0
        torch.cuda.synchronize()
        # the same kernels in the same order: bitwise equal
        assert float(n_na.item()) == n_ref
        kind = S.export_level(level)[0]
        act = torch.tensor(np.pad(kind != 0, 2), device="cuda")
        assert torch.equal(r_na[act], r_ref[act])
    S.close()


def test_noalloc_rejects_bad_arguments():
    _torch()
    import paper_2601_02975_amd as mg
    P = W.unit_disk_config(0, 64)
    S = mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps)
    lib = mg.lib()
    lib.mg_residual_norm_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.mg_residual_norm_noalloc(S.h, 0, None, None, None, None, None) == -1
    assert lib.mg_residual_norm_noalloc(S.h, 99, None, None, None, None, None) == -1
    S.close()
