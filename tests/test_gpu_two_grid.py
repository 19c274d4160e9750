"""Two-grid analysis on the GPU (eq. (5.10)): with two levels the V-cycle on
b = 0 is the two-grid error operator TG = T^nu2 (I - P A_c^{-1} R A) T^nu1,
so ARPACK on the GPU's V-cycle gives rho(TG).  Pinned to Table 1 of the
paper (unit square, (a,b,c) = (1,0,2), omega = 1/2) to its printed digits."""
import numpy as np
import pytest

import workloads as W
from conftest import golden

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_table1_two_grid_radius_on_gpu():
    import scipy.sparse.linalg as spla
    torch = _torch()
    import paper_2601_02975_amd as mg
    P = W.unit_square_config(64)
    for nu1, nu2, rho in golden("table1_unit_square_rho.txt"):
        S = mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, nu=(int(nu1), int(nu2)), n_levels=2)
        kind = S.export_level(0)[0].reshape(P.grid.ny, P.grid.nx)
        jj, ii = np.nonzero(kind > 0)
        n = len(ii)
        pad = (P.grid.ny + 4, P.grid.nx + 4)
        zero = torch.zeros(pad, dtype=torch.float64, device="cuda")

        def tg(x):
            u = np.zeros(pad)
            u[jj + 2, ii + 2] = np.real(x)
            ud = torch.tensor(u, device="cuda")
            S.vcycle(zero, ud)
            return ud.cpu().numpy()[jj + 2, ii + 2]

        T = spla.LinearOperator((n, n), matvec=tg, dtype=np.float64)
        ev = spla.eigs(T, k=3, which="LM", return_eigenvectors=False, maxiter=5000, tol=1e-8)
        got = max(abs(ev))
        print("nu = (%d, %d): rho(TG) %.4f (Table 1: %.3f)" % (nu1, nu2, got, rho))
        assert got == pytest.approx(rho, abs=6e-4)
        S.close()
