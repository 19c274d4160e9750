"""The multicolour variant of the smoother (an extension; the paper's
smoother is the omega-Jacobi of eq. (5.5)): one launch per sweep updates the
SFV cells colour by colour inside each LDS tile of 64 x 16 cells (FP64),
with the values at the start of the sweep across tiles and in ghost cells.
The oracle defines the same sweep with those blocks, so FP64 sweeps are
compared per level; solves are compared at convergence with the Jacobi
path's solution, in both precisions."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import CASES, FP64_PARITY, _torch, from_dev, rel, to_dev

pytestmark = pytest.mark.gpu


def _oracle_mc(name):
    from oracle.multigrid import Hierarchy
    P = CASES[name]()
    return P, Hierarchy(P.grid, P.curves, P.a, P.b, P.c, P.eps, colouring=True, block=(64, 16))


@pytest.mark.parametrize("name", ["disk64", "three_disks128", "star128", "square_cross32"])
def test_multicolour_sweep_parity(name):
    import paper_2601_02975_amd as mg
    P, H = _oracle_mc(name)
    S = mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, colouring=mg.SMOOTH_MULTICOLOUR)
    rng = np.random.default_rng(31)
    for l, L in enumerate(H.levels):
        u = rng.standard_normal(L.n)
        b = rng.standard_normal(L.n) / (L.h * L.h)
        want = H.smooth(l, u, b)
        ud = to_dev(L, u)
        S.smooth(l, to_dev(L, b), ud)
        err = rel(from_dev(L, ud), want)
        bound = FP64_PARITY
        print("level %d multicolour sweep rel diff %.2e (bound %.1e)" % (l, err, bound))
        assert err <= bound
    S.close()


@pytest.mark.parametrize("name", ["disk64", "three_disks128", "star128"])
@pytest.mark.parametrize("precision", [0, 1])
def test_multicolour_solve_converges_to_the_same_solution(name, precision):
    torch = _torch()
    import paper_2601_02975_amd as mg
    P = CASES[name]()
    J = mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=precision)
    C = mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=precision,
                  colouring=mg.SMOOTH_MULTICOLOUR)
    f, g = J.project(P.solution)
    uj, uc = torch.zeros_like(f), torch.zeros_like(f)
    itj, relj, cj = J.solve(f, g, uj, 1e-11)
    itc, relc, cc = C.solve(f, g, uc, 1e-11)
    d = float((uc - uj).abs().max() / uj.abs().max())
    print("Jacobi %d cycles, multicolour %d cycles, solutions differ by %.2e" % (itj, itc, d))
    assert cj == 0 and cc == 0 and relc <= 1e-11
    # both iterates are within |A^-1| 1e-11 |b| of u*: a few 1e-9 relative
    assert d <= 1e-8
    J.close()
    C.close()
