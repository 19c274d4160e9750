"""Pins of the oracle's discretisation and multigrid solver against values the
paper prints (Tables 1 and 2), polynomial exactness and direct solves."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from conftest import golden
from oracle.discretize import Level, PLG, SFV
from oracle.multigrid import Hierarchy
from oracle.rhs import cell_averages, rhs

POLY4 = {(0, 0): 0.3, (1, 0): -0.7, (0, 1): 0.2, (2, 0): 0.5, (1, 1): -0.4, (0, 2): 0.9, (3, 0): 0.25,
         (2, 1): -0.6, (1, 2): 0.35, (0, 3): -0.45, (4, 0): 0.15, (3, 1): 0.55, (2, 2): -0.3,
         (1, 3): 0.2, (0, 4): -0.1}
POLY3 = {k: v for k, v in POLY4.items() if sum(k) <= 3}


def _errors(level, u, uexact):
    e = u - uexact
    vol = level.cg.volfrac[level.cells_j, level.cells_i]
    return (np.abs(e).max(), float(np.sum(vol * np.abs(e)) / vol.sum()),
            math.sqrt(float(np.sum(vol * e * e) / vol.sum())))


@pytest.mark.parametrize("row", [0, 1])
def test_table2_unit_square_errors(row):
    """Section 6.1, Table 2: errors of the exact discrete solution on the
    unit square, to the three printed digits."""
    n, linf, l1, l2 = golden("table2_unit_square.txt")[row]
    P = W.unit_square_config(int(n))
    L = Level(P.grid, P.curves, P.a, P.b, P.c, P.eps)
    assert not L.is_plg.any()
    b, _, _ = rhs(L, P.solution)
    u = spla.spsolve(L.A.tocsc(), b)
    got = _errors(L, u, cell_averages(L, P.solution.u))
    for g, want in zip(got, (linf, l1, l2)):
        assert float("%.2e" % g) == pytest.approx(want, rel=0.006)


def test_table1_two_grid_radius_unit_square():
    """Section 5.3, Table 1: spectral radius of TG on the unit square, all
    five (nu1, nu2) pairs, three printed digits (h = 1/64 over 1/32)."""
    P = W.unit_square_config(64)
    H = Hierarchy(P.grid, P.curves, P.a, P.b, P.c, P.eps, n_levels=2)
    for nu1, nu2, rho in golden("table1_unit_square_rho.txt"):
        T = H.two_grid_operator(int(nu1), int(nu2))
        ev = spla.eigs(T, k=3, which="LM", return_eigenvectors=False, maxiter=5000, tol=1e-8)
        assert max(abs(ev)) == pytest.approx(rho, abs=6e-4)


def _poly_problem(base, coeffs):
    P = base
    return W.Problem(P.name, P.grid, P.curves, P.a, P.b, P.c, W.Poly(coeffs, P.a, P.b, P.c), P.eps)


def _robin_box(base, alpha1=1.0, alpha2=0.5):
    """base with Robin (alpha1, alpha2) on every box side."""
    box = W.box_curve(0.0, 0.0, 1.0, 1.0, W.BC_ROBIN, alpha1, alpha2)
    return W.Problem(base.name + "_robin_box", base.grid, [box] + list(base.curves[1:]), base.a, base.b, base.c,
                     base.solution, base.eps)


@pytest.mark.parametrize("maker,n,coeffs", [
    (W.unit_disk_config, 64, POLY4),
    (W.three_disks_config, 128, POLY3),
    (W.star_config, 128, POLY3),
    (lambda s, n: W.unit_square_config(n, 1.0, 0.5, 2.0), 32, POLY3),
    (lambda s, n: _robin_box(W.unit_disk_config(s, n)), 64, POLY4),
    (lambda s, n: _robin_box(W.unit_square_config(n, 1.0, 0.5, 2.0), 2.0, 0.25), 32, POLY3),
    (W.bezier_config, 96, POLY3),
])
def test_polynomial_solution_is_exact(maker, n, coeffs):
    """Every row is exact on the polynomials it must reproduce (degree 4 for
    eq. (4.7) and the PLG fits; the corner ghosts of the cross term are exact
    to degree 3), so the discrete solution equals the exact cell averages."""
    P = _poly_problem(maker(0, n), coeffs)
    L = Level(P.grid, P.curves, P.a, P.b, P.c, P.eps)
    b, _, _ = rhs(L, P.solution)
    ue = cell_averages(L, P.solution.u)
    tau = L.A @ ue - b
    assert np.abs(tau).max() <= 1e-9 * np.abs(b).max()
    u = spla.spsolve(L.A.tocsc(), b)
    assert np.abs(u - ue).max() <= 1e-9 * np.abs(ue).max()


def test_plg_rows_exact_on_pi4_and_weighted_min_norm():
    """eqs. (4.14)-(4.18): M beta = phibar, and W^{-1} beta lies in the row
    space of M (the optimality condition of the weighted minimum-norm
    problem, Lemma 4.4)."""
    P = W.unit_disk_config(0, 64)
    L = Level(P.grid, P.curves, P.a, P.b, P.c, P.eps)
    checked = 0
    for (i, j), (beta, bb) in L.beta.items():
        lat = L.lattice[(i, j)]
        M = np.array([L._avg_monomials((i + d[0], j + d[1]), d) for d in lat]).T
        w = np.array([max(math.hypot(*d), 0.5) for d in lat])
        full = beta
        if bb is not None:
            M = np.hstack([M, L.boundary_average_of_basis(i, j)[:, None]])
            w = np.append(w, 0.5)
            full = np.append(beta, bb)
            # W^{-1} beta = M^T y for some y
            y = np.linalg.lstsq(M.T, w * full, rcond=None)[0]
            assert np.abs(M.T @ y - w * full).max() <= 1e-8 * np.abs(w * full).max()
        phibar = L._lphi(i, j)
        assert np.abs(M @ full - phibar).max() <= 1e-10 * np.abs(phibar).max()
        checked += 1
    assert checked == int(L.is_plg.sum())


@pytest.fixture(scope="module")
def disk_hierarchy():
    P = W.unit_disk_config(3, 64)
    H = Hierarchy(P.grid, P.curves, P.a, P.b, P.c, P.eps)
    b, _, _ = rhs(H.levels[0], P.solution)
    return P, H, b


def test_block_smoother_zeroes_plg_residual(disk_hierarchy):
    """After one block-smoother sweep r2 = 0 (Definition 5.6)."""
    P, H, b = disk_hierarchy
    L = H.levels[0]
    u = H.smooth(0, np.random.default_rng(1).standard_normal(L.n), b)
    r = b - L.A @ u
    assert np.abs(r[L.is_plg]).max() <= 1e-10 * np.abs(b).max()
    assert np.abs(r[~L.is_plg]).max() > 1e-3 * np.abs(b).max()


def test_vcycle_converges_to_direct_solution(disk_hierarchy):
    """The V-cycle iteration converges to u* = A^{-1} b (eq. (4.19))."""
    P, H, b = disk_hierarchy
    A = H.levels[0].A
    u, it, rel = H.solve(b, tol=1e-12, max_iters=60)
    ustar = spla.spsolve(A.tocsc(), b)
    assert rel <= 1e-12
    assert np.abs(u - ustar).max() <= 1e-10 * np.abs(ustar).max()


def test_vcycle_is_affine(disk_hierarchy):
    """Vcycle(u, b) = u + Vcycle(0, b - A u): the defect-correction form used
    by the mixed-precision path equals Algorithm 3 in exact arithmetic."""
    P, H, b = disk_hierarchy
    L = H.levels[0]
    u0 = np.random.default_rng(2).standard_normal(L.n)
    v1 = H.vcycle(0, u0, b)
    v2 = u0 + H.vcycle(0, np.zeros(L.n), b - L.A @ u0)
    assert np.abs(v1 - v2).max() <= 1e-9 * np.abs(v1).max()


def test_fourth_order_convergence_disk():
    """Solution error ratio near 16 per halving of h (Tables 2-5 behaviour)."""
    errs = []
    for n in (64, 128):
        P = W.unit_disk_config(0, n)
        L = Level(P.grid, P.curves, P.a, P.b, P.c, P.eps)
        b, _, _ = rhs(L, P.solution)
        u = spla.spsolve(L.A.tocsc(), b)
        errs.append(np.abs(u - cell_averages(L, P.solution.u)).max())
    assert errs[0] / errs[1] > 8.0


def test_fmg_converges_to_direct_solution(disk_hierarchy):
    """FMG cycles on residual equations (Algorithm 4, Sec. 5.4) converge to
    the same discrete solution u* = A^{-1} b as the direct solve."""
    P, H, b = disk_hierarchy
    L = H.levels[0]
    direct = spla.spsolve(L.A.tocsc(), b)
    u, it, rel = H.solve(b, tol=1e-12, max_iters=60, cycle="FMG")
    assert rel <= 1e-12
    assert np.abs(u - direct).max() <= 1e-9 * np.abs(direct).max()


def test_fmg_factor_is_h_independent_and_beats_vcycle():
    """Averaged residual reduction of the FMG iteration on the unit square,
    (a,b,c) = (1,0,2), nu = (3,3): independent of h (Sec. 5.4: O(1) cycles)
    and better than the V-cycle's, which grows with the depth here."""
    factors = {}
    for n in (64, 128):
        P = W.unit_square_config(n, 1.0, 0.0, 2.0)
        H = Hierarchy(P.grid, P.curves, P.a, P.b, P.c, P.eps)
        b, _, _ = rhs(H.levels[0], P.solution)
        for cyc in ("V", "FMG"):
            hist = []
            H.solve(b, tol=1e-11, max_iters=80, history=hist, cycle=cyc)
            rels = [r for _, r in hist]
            factors[(n, cyc)] = (rels[-1] / rels[0]) ** (1.0 / (len(rels) - 1))
    assert abs(factors[(64, "FMG")] - factors[(128, "FMG")]) <= 0.05
    assert factors[(128, "FMG")] < factors[(128, "V")]
    assert factors[(128, "FMG")] < 0.5


def _averaged_factor(H, b, tol, cycle="V", max_iters=120):
    """(||r_N|| / ||r_0||)^(1/N) over the N cycles from u = 0 to tol (the
    relative L-inf residual of Sec. 6.5)."""
    hist = []
    H.solve(b, tol=tol, max_iters=max_iters, history=hist, cycle=cycle)
    return hist[-1][1] ** (1.0 / len(hist))


def test_two_level_vcycle_factor_is_h_independent_and_matches_table7():
    """With two levels the V-cycle is the two-grid cycle, whose spectral
    radius Table 1 shows to be h-independent; its averaged residual reduction
    is h-independent too (spread <= 0.01 over h = 1/32 .. 1/128), and for
    nu = (3, 3) it is Table 7's unit-square V-cycle value 0.330 (to 0.01)."""
    f = {}
    for n in (32, 64, 128):
        P = W.unit_square_config(n, 1.0, 0.0, 2.0)
        H = Hierarchy(P.grid, P.curves, P.a, P.b, P.c, P.eps, n_levels=2, nu=(3, 3))
        b, _, _ = rhs(H.levels[0], P.solution)
        f[n] = _averaged_factor(H, b, 1e-12)
    assert max(f.values()) - min(f.values()) <= 0.01
    assert f[128] == pytest.approx(0.330, abs=0.01)


def test_two_level_vcycle_spectral_radius_is_table1():
    """The V-cycle code itself (not the separate TG operator) with two levels
    and b = 0 is the error propagation of eq. (5.10): its spectral radius is
    Table 1's for (2, 1) and (3, 3)."""
    P = W.unit_square_config(64)
    want = {(int(a), int(c)): rho for a, c, rho in golden("table1_unit_square_rho.txt")}
    for nu in ((2, 1), (3, 3)):
        H = Hierarchy(P.grid, P.curves, P.a, P.b, P.c, P.eps, n_levels=2, nu=nu)
        n = H.levels[0].n
        zero = np.zeros(n)
        op = spla.LinearOperator((n, n), matvec=lambda e: H.vcycle(0, np.asarray(e).ravel(), zero), dtype=float)
        ev = spla.eigs(op, k=3, which="LM", return_eigenvectors=False, maxiter=5000, tol=1e-8)
        assert max(abs(ev)) == pytest.approx(want[nu], abs=6e-4)


def _error_propagation(H, l, v):
    """E_l v for Algorithm 3 on level l, by the textbook recursion for a
    V-cycle with a zero coarse initial guess:
        E_l = S^nu2 (I - P (I - E_{l+1}) A_{l+1}^{-1} R A_l) S^nu1,
    E_bottom = 0, where S is the smoother's error propagation (eq. (5.4)
    with b = 0) and the coarse inverse is a sparse direct solve."""
    if l == len(H.levels) - 1:
        return np.zeros_like(v)
    zero = np.zeros_like(v)
    for _ in range(H.nu1):
        v = H.smooth(l, v, zero)
    rc = H.R[l] @ (H.levels[l].A @ v)
    xc = spla.spsolve(H.levels[l + 1].A.tocsc(), rc)
    v = v - H.P[l] @ (xc - _error_propagation(H, l + 1, xc))
    for _ in range(H.nu2):
        v = H.smooth(l, v, zero)
    return v


def _fmg_operator(H, l, r):
    """The map r -> FMG(A_l, r) of Algorithm 4, built from the V-cycle's
    error propagation: the V-cycle started from e0 returns
    e0 + (I - E_l)(A_l^{-1} r - e0), so
        F_l r = E_l P F_{l+1} R r + (I - E_l) A_l^{-1} r,  F_bottom = A^{-1}."""
    A = H.levels[l].A
    x = spla.spsolve(A.tocsc(), r)
    if l == len(H.levels) - 1:
        return x
    e0 = H.P[l] @ _fmg_operator(H, l + 1, H.R[l] @ r)
    return e0 + (x - e0) - _error_propagation(H, l, x - e0)


@pytest.fixture(scope="module")
def disk_three_levels():
    P = W.unit_disk_config(0, 64)
    H = Hierarchy(P.grid, P.curves, P.a, P.b, P.c, P.eps, n_levels=3, nu=(2, 1))
    assert H.levels[1].is_plg.any() and H.levels[2].is_plg.any()
    return H


def test_vcycle_is_the_multilevel_error_recursion(disk_three_levels):
    """Algorithm 3 on three levels with PLG cells on every level, nu = (2, 1):
    Vcycle(u, b) - u* = E (u - u*) with u* = A^{-1} b and E from the
    recursion above (catches a wrong coarse initial guess, restricting b
    instead of the residual, a sign or an exchanged nu1/nu2)."""
    H = disk_three_levels
    A = H.levels[0].A
    rng = np.random.default_rng(5)
    u = rng.standard_normal(A.shape[0])
    b = rng.standard_normal(A.shape[0])
    ustar = spla.spsolve(A.tocsc(), b)
    got = H.vcycle(0, u, b) - ustar
    want = _error_propagation(H, 0, u - ustar)
    assert np.abs(got - want).max() <= 1e-9 * np.abs(u - ustar).max()


def test_fmg_is_the_nested_vcycle_operator(disk_three_levels):
    """Algorithm 4 on the same hierarchy equals F_0 r from the V-cycle's
    error propagation (restriction of r, bottom solve, interpolation as the
    initial guess, V-cycle on the residual equation)."""
    H = disk_three_levels
    r = np.random.default_rng(6).standard_normal(H.levels[0].n)
    got = H.fmg(0, r)
    want = _fmg_operator(H, 0, r)
    assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()


def test_robin_box_vcycle_converges_to_direct_solution():
    """Robin (1, 0.5) on all four box sides (ghosts from the Robin reading of
    Sec. 4.1), the disk hole Dirichlet: the V-cycle iteration converges to
    the direct solve of the assembled system."""
    P = _robin_box(W.unit_disk_config(0, 64))
    H = Hierarchy(P.grid, P.curves, P.a, P.b, P.c, P.eps)
    b, _, _ = rhs(H.levels[0], P.solution)
    direct = spla.spsolve(H.levels[0].A.tocsc(), b)
    u, it, rel = H.solve(b, tol=1e-12, max_iters=100)
    assert rel <= 1e-12
    assert np.abs(u - direct).max() <= 1e-9 * np.abs(direct).max()


# -- the multicolour variant of the smoother (an extension, not in the paper) --

@pytest.fixture(scope="module")
def mc_hierarchies():
    P = W.three_disks_config(0, 128)
    H = Hierarchy(P.grid, P.curves, P.a, P.b, P.c, P.eps, n_levels=2, colouring=True, block=(64, 16))
    Q = W.unit_disk_config(0, 64)
    G = Hierarchy(Q.grid, Q.curves, Q.a, Q.b, Q.c, Q.eps, n_levels=2, colouring=True, block=(64, 16))
    return (P, H), (Q, G)


def test_multicolour_colours_are_independent(mc_hierarchies):
    """No two SFV cells of one colour couple through the in-block stencil:
    (i + 3j) mod 9 for the 5 x 5 box (b != 0), (i + j) mod 3 for the plus
    shape (b = 0), so each colour is a Jacobi step on independent cells."""
    for P, H in mc_hierarchies:
        for l in range(len(H.levels)):
            colour, a_in = H.sm[l][8], H.sm[l][9]
            for k in range(int(colour.max()) + 1):
                sel = np.nonzero(colour == k)[0]
                blk = a_in[sel][:, sel].tocoo()
                assert np.all(blk.row == blk.col)


def test_multicolour_reduces_to_jacobi_with_one_cell_blocks(mc_hierarchies):
    """With blocks of a single cell every neighbour comes from the sweep's
    starting values: the multicolour sweep is the omega-Jacobi sweep of
    eq. (5.5) (then the PLG solve)."""
    (P, H), _ = mc_hierarchies
    J = Hierarchy(P.grid, P.curves, P.a, P.b, P.c, P.eps, n_levels=2)
    C = Hierarchy(P.grid, P.curves, P.a, P.b, P.c, P.eps, n_levels=2, colouring=True, block=(1, 1))
    rng = np.random.default_rng(8)
    n = J.levels[0].n
    u, b = rng.standard_normal(n), rng.standard_normal(n)
    assert np.abs(C.smooth(0, u, b) - J.smooth(0, u, b)).max() <= 1e-12 * np.abs(J.smooth(0, u, b)).max()


def test_multicolour_fixed_point_is_the_solution(mc_hierarchies):
    """u* = A^{-1} b is left unchanged by a multicolour sweep (every partial
    residual it uses is that of u*), and the sweep changes any other u."""
    for P, H in mc_hierarchies:
        L = H.levels[0]
        b = np.random.default_rng(9).standard_normal(L.n)
        ustar = spla.spsolve(L.A.tocsc(), b)
        assert np.abs(H.smooth(0, ustar, b) - ustar).max() <= 1e-9 * np.abs(ustar).max()
        v = ustar + np.random.default_rng(10).standard_normal(L.n)
        assert np.abs(H.smooth(0, v, b) - v).max() > 1e-3


# -- periodic box sides (Sec. 4.1) ---------------------------------------------

def _periodic_square(n, a=1.0, b=0.5, c=2.0):
    box = W.box_curve(0.0, 0.0, 1.0, 1.0)
    box = [W.Segment(s.kind, s.p, W.BC_PERIODIC if k in (1, 3) else W.BC_DIRICHLET) for k, s in enumerate(box)]
    return Level(W.Grid(0.0, 0.0, 1.0 / n, n, n), [box], a, b, c, 0.1)


def test_periodic_operator_commutes_with_the_cyclic_shift():
    """On the unit square periodic in x (Dirichlet in y, cross term), the
    discrete operator commutes with a shift by one cell in x, including the
    rows next to the periodic sides (a wrong wrap index would not)."""
    L = _periodic_square(32)
    rng = np.random.default_rng(3)
    u = rng.standard_normal((L.ny, L.nx))
    Au = (L.A @ u[L.cells_j, L.cells_i])
    v = np.roll(u, 1, axis=1)
    Av = L.A @ v[L.cells_j, L.cells_i]
    grid = np.zeros((L.ny, L.nx))
    grid[L.cells_j, L.cells_i] = Au
    assert np.abs(Av - np.roll(grid, 1, axis=1)[L.cells_j, L.cells_i]).max() <= 1e-10 * np.abs(Au).max()


def test_periodic_fourth_order_convergence_and_vcycle():
    """A disk hole in a box periodic in x: solution error ratio near 16 per
    halving of h (4th order), and the V-cycle converges to the direct solve."""
    errs = []
    for n in (64, 128):
        P = W.periodic_config(0, n)
        L = Level(P.grid, P.curves, P.a, P.b, P.c, P.eps)
        b, _, _ = rhs(L, P.solution)
        u = spla.spsolve(L.A.tocsc(), b)
        errs.append(np.abs(u - cell_averages(L, P.solution.u)).max())
    assert errs[0] / errs[1] > 12.0
    P = W.periodic_config(0, 64)
    H = Hierarchy(P.grid, P.curves, P.a, P.b, P.c, P.eps, nu=(4, 4))
    b, _, _ = rhs(H.levels[0], P.solution)
    ustar = spla.spsolve(H.levels[0].A.tocsc(), b)
    u, it, rel = H.solve(b, tol=1e-12, max_iters=100)
    assert rel <= 1e-12 and np.abs(u - ustar).max() <= 1e-10 * np.abs(ustar).max()


def test_periodic_sides_must_pair():
    from oracle.geometry import GeometryError
    box = W.box_curve(0.0, 0.0, 1.0, 1.0)
    box[1] = W.Segment("line", box[1].p, W.BC_PERIODIC)
    with pytest.raises(GeometryError):
        Level(W.Grid(0.0, 0.0, 1.0 / 32, 32, 32), [box], 1.0, 0.0, 1.0, 0.1)
