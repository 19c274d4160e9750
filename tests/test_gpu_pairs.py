"""Two-sweep tiles against the FP64 oracle.

On levels whose launch A is split, consecutive Jacobi sweeps run in pairs,
and the tiles whose cells and 2-cell halo are SFV cells (4-cell halo inside
the box) do both sweeps' SFV updates in one pass; the other tiles, the PLG
groups and launch B run once per sweep.  A 64-cell-wide tile needs its
4-cell halo inside the box, so the small oracle cases have no such tile:
these cases are 256^2, with every level split.  nu = (3, 3) runs one pair
and one single sweep on each side of the cycle; the mixed-precision solve
starts its FP32 cycles from zero (the pair path's zero-iterate branch).
"""
import functools

import numpy as np
import pytest

import workloads as W
from test_gpu_parity import FP64_PARITY, _torch, from_dev, rel, to_dev

pytestmark = pytest.mark.gpu

EPS64 = np.finfo(np.float64).eps

CASES = {
    "disk256": lambda: W.unit_disk_config(0, 256),          # b = 0: the 13-point stencil
    "three_disks256": lambda: W.three_disks_config(0, 256),  # b != 0: the 25-point stencil
}


@functools.lru_cache(maxsize=None)
def oracle(name):
    from oracle.multigrid import Hierarchy
    P = CASES[name]()
    return P, Hierarchy(P.grid, P.curves, P.a, P.b, P.c, P.eps, nu=(3, 3))


@functools.lru_cache(maxsize=None)
def product(name, pairs, precision=0, nu=(3, 3)):
    import paper_2601_02975_amd as mg
    P = CASES[name]()
    return mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=precision, nu=nu, max_iters=200,
                     split_cells=1, pair_sweeps=0 if pairs else -1)


@pytest.mark.parametrize("name", list(CASES))
def test_pair_tiles_exist(name):
    S = product(name, True)
    n_pair, n_sfv = S.info["n_pair_sfv"], S.info["n_sfv"]
    print("%s: two-sweep SFV cells per level %s of %s" % (name, n_pair, n_sfv))
    assert 0 < n_pair[0] < n_sfv[0]
    assert product(name, False).info["n_pair_sfv"][0] == 0


@pytest.mark.parametrize("name", list(CASES))
def test_pair_vcycle_iterates_match_oracle(name):
    """u_k of Algorithm 3 (nu = (3, 3)) from u_0 = 0, k = 1..3, FP64."""
    from oracle.rhs import rhs
    P, H = oracle(name)
    S = product(name, True)
    L = H.levels[0]
    b, _, _ = rhs(L, P.solution)
    bd = to_dev(L, b)
    uo = np.zeros(L.n)
    ud = to_dev(L, uo)
    for l in range(len(H.levels)):
        assert 4 * EPS64 * max(1.0, S.info["cond_A22"][l]) <= FP64_PARITY
    for k in range(3):
        uo = H.vcycle(0, uo, b)
        S.vcycle(bd, ud)
        err = rel(from_dev(L, ud), uo)
        print("%s iterate %d: rel diff %.2e" % (name, k + 1, err))
        assert err <= FP64_PARITY


@pytest.mark.parametrize("nu", [(2, 2), (3, 3), (2, 1)])
@pytest.mark.parametrize("name", list(CASES))
def test_pairs_on_and_off_agree(name, nu):
    """Each cell's update is the same expression in both paths; with the
    mixed term (b != 0) the compiler may contract the 25-point sums into
    fused multiply-adds differently in the two kernels, so the iterates
    agree to rounding (bitwise where b = 0)."""
    torch = _torch()
    from oracle.rhs import rhs
    P, H = oracle(name)
    L = H.levels[0]
    b, _, _ = rhs(L, P.solution)
    bd = to_dev(L, b)
    S1, S0 = product(name, True, nu=nu), product(name, False, nu=nu)
    u1, u0 = to_dev(L, np.zeros(L.n)), to_dev(L, np.zeros(L.n))
    for k in range(3):
        S1.vcycle(bd, u1)
        S0.vcycle(bd, u0)
        torch.cuda.synchronize()
        err = rel(from_dev(L, u1), from_dev(L, u0))
        print("%s nu %s iterate %d: pairs on/off rel diff %.2e" % (name, nu, k + 1, err))
        if P.b == 0.0:
            assert err == 0.0
        assert err <= 1e-13


@pytest.mark.parametrize("name", list(CASES))
def test_pair_mixed_solve(name):
    """Mixed-precision solves (FP32 V-cycles from zero) with and without
    pairs: the same iteration count, the same solution to rounding."""
    torch = _torch()
    P, H = oracle(name)
    L = H.levels[0]
    S1, S0 = product(name, True, precision=1), product(name, False, precision=1)
    f, g = S1.project(P.solution, 8)
    u1, u0 = torch.zeros_like(f), torch.zeros_like(f)
    it1, r1, c1 = S1.solve(f, g, u1, 1e-10)
    it0, r0, c0 = S0.solve(f, g, u0, 1e-10)
    err = float((u1 - u0).abs().max() / u0.abs().max())
    print("%s: %d / %d iterations, rel residual %.2e / %.2e, solutions differ by %.2e" % (
        name, it1, it0, r1, r0, err))
    assert c1 == 0 and c0 == 0 and it1 == it0
    assert err <= 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_pair_fmg_solve(name):
    """FMG cycles in FP64 (Algorithm 4 on residual equations: the finest
    level's V-cycle starts from the interpolant, its buffers rotate with the
    residual equation's) with and without pairs."""
    torch = _torch()
    import paper_2601_02975_amd as mg
    P, H = oracle(name)
    sol = []
    for pairs in (True, False):
        S = mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=mg.FP64, nu=(2, 2), max_iters=200,
                      cycle=mg.CYCLE_FMG, split_cells=1, pair_sweeps=0 if pairs else -1)
        f, g = S.project(P.solution, 8)
        u = torch.zeros_like(f)
        it, r, c = S.solve(f, g, u, 1e-10)
        assert c == 0
        sol.append((it, u))
        S.close()
    err = float((sol[0][1] - sol[1][1]).abs().max() / sol[1][1].abs().max())
    print("%s FMG: %d / %d cycles, solutions differ by %.2e" % (name, sol[0][0], sol[1][0], err))
    assert sol[0][0] == sol[1][0] and err <= 1e-12
