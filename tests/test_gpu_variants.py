"""Every launch shape of the smoother against the FP64 oracle, FP32 steps
against their FP64 definitions, the transfer steps, and the conditioning the
library reports for A22.

The launch shapes (split launch A, 8- or 32-row tiles, split launch B) are
chosen by grid size in production; the options force each of them on the
small oracle cases here, so that no kernel variant is checked only at sizes
the oracle cannot reach.  Bounds: the SFV rows of a sweep are sums of at most
25 products (a few units of roundoff); the PLG rows come from an exact solve
with A22 by a different method (segment inverses and a Schur complement here,
a sparse LU in the oracle), whose difference is bounded by cond(A22) times
the unit roundoff, with cond(A22) the estimate the library reports.
"""
import functools

import numpy as np
import pytest

import workloads as W
from test_gpu_parity import CASES, FP64_PARITY, _torch, from_dev, oracle, rel, to_dev

pytestmark = pytest.mark.gpu

EPS64 = np.finfo(np.float64).eps
EPS32 = np.finfo(np.float32).eps

# launch shapes: every level split into a tile kernel and PLG groups (the
# FP64 16-row and FP32 32-row tile kernels and the PLG groups that read the
# tiles' output), fused launches with 32-row tiles everywhere, fused with
# 8-row tiles everywhere; each with launch B in two kernels wherever there
# are separators
SHAPES = {
    "split_a": dict(split_cells=1, split_b_sep=1),
    "fused_tall": dict(split_cells=1 << 40, small_cells=-1, split_b_sep=1),
    "fused_short": dict(split_cells=1 << 40, small_cells=1 << 40, split_b_sep=1),
}


@functools.lru_cache(maxsize=None)
def product(name, shape, precision=0, nu=(3, 3)):
    import paper_2601_02975_amd as mg
    P = CASES[name]()
    return mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=precision, nu=nu, **SHAPES[shape])


def sweep_bound(S, l):
    """A sweep's PLG rows differ by about cond(A22) eps; the parity target
    1e-12 holds while cond(A22) stays below ~1e3 (checked)."""
    b = 4 * EPS64 * max(1.0, S.info["cond_A22"][l])
    assert b <= FP64_PARITY
    return FP64_PARITY


@pytest.mark.parametrize("shape", list(SHAPES))
@pytest.mark.parametrize("name", ["disk64", "three_disks128", "star128", "square_cross32"])
def test_sweep_parity_every_shape(name, shape):
    """One FP64 block-smoother sweep (Definition 5.6) on every level."""
    P, H = oracle(name)
    S = product(name, shape)
    rng = np.random.default_rng(21)
    for l, L in enumerate(H.levels):
        u = rng.standard_normal(L.n)
        b = rng.standard_normal(L.n) / (L.h * L.h)
        want = H.smooth(l, u, b)
        ud = to_dev(L, u)
        S.smooth(l, to_dev(L, b), ud)
        err = rel(from_dev(L, ud), want)
        print("%s level %d (%dx%d, %d separators): rel diff %.2e, bound %.1e" % (
            shape, l, L.nx, L.ny, S.info["n_sep"][l], err, sweep_bound(S, l)))
        assert err <= sweep_bound(S, l)


@pytest.mark.parametrize("shape", list(SHAPES))
@pytest.mark.parametrize("name", ["disk64", "three_disks128", "star128"])
def test_vcycle_iterates_every_shape(name, shape):
    """u_k of Algorithm 3 from u_0 = 0, k = 1..4, FP64."""
    from oracle.rhs import rhs
    P, H = oracle(name)
    S = product(name, shape)
    L = H.levels[0]
    b, _, _ = rhs(L, P.solution)
    bd = to_dev(L, b)
    uo = np.zeros(L.n)
    ud = to_dev(L, uo)
    bound = max(sweep_bound(S, l) for l in range(len(H.levels)))
    for k in range(4):
        uo = H.vcycle(0, uo, b)
        S.vcycle(bd, ud)
        err = rel(from_dev(L, ud), uo)
        print("%s iterate %d rel diff %.2e (bound %.1e)" % (shape, k + 1, err, bound))
        assert err <= bound


@pytest.mark.parametrize("name", ["disk64", "three_disks128", "star128", "square_cross32"])
def test_transfers_parity(name):
    """Restriction of the residual (eq. (5.8)) with every residual computed,
    and the piecewise-constant correction (eq. (5.9)), FP64, every level."""
    torch = _torch()
    P, H = oracle(name)
    S = product(name, "split_a")
    rng = np.random.default_rng(22)
    for l in range(len(H.levels) - 1):
        L, C = H.levels[l], H.levels[l + 1]
        u = rng.standard_normal(L.n)
        b = rng.standard_normal(L.n) / (L.h * L.h)
        want = H.R[l] @ (b - L.A @ u)
        bc = to_dev(C, np.zeros(C.n))
        S.restrict(l, to_dev(L, b), to_dev(L, u), bc)
        # rounding of the residual sums and of the quarter-sums of children
        au = H.R[l] @ (np.abs(b) + abs(L.A) @ np.abs(u))
        got = from_dev(C, bc)
        assert np.all(np.abs(got - want) <= 32 * EPS64 * au + 1e-12 * np.abs(want).max())
        ec = rng.standard_normal(C.n)
        want = u + H.P[l] @ ec
        ud = to_dev(L, u)
        S.prolong(l, to_dev(C, ec), ud)
        assert np.all(np.abs(from_dev(L, ud) - want) <= 2 * EPS64 * (np.abs(u) + np.abs(H.P[l] @ ec)))


@pytest.mark.parametrize("name", ["disk64", "three_disks128", "star128", "square_cross32"])
def test_fp32_steps_against_fp64_definitions(name):
    """The FP32 kernels of the mixed-precision V-cycle, step by step on every
    level, against the oracle's FP64 steps on the same (FP32-representable)
    inputs: one sweep, one restriction and one correction.  Bound: FP32
    rounding of the stencil sums (32 eps32 of |u| + (omega/|D|)(|b| + |A||u|)
    on SFV rows) and of the exact A22 solve (cond(A22) times that, on PLG
    rows)."""
    torch = _torch()
    P, H = oracle(name)
    S = product(name, "split_a", precision=1)
    rng = np.random.default_rng(23)
    f32 = lambda v: v.astype(np.float32).astype(np.float64)
    dev32 = lambda L, v: to_dev(L, v).to(torch.float32)
    back = lambda L, t: from_dev(L, t.to(torch.float64))
    for l, L in enumerate(H.levels):
        u = f32(rng.standard_normal(L.n))
        b = f32(rng.standard_normal(L.n) / (L.h * L.h))
        want = H.smooth(l, u, b)
        ud = dev32(L, u)
        S.smooth32(l, dev32(L, b), ud)
        got = back(L, ud)
        d = 2.5 * (L.a + L.c) / (L.h * L.h)
        scale = np.abs(u) + H.omega / d * (np.abs(b) + abs(L.A) @ np.abs(u))
        tol = 32 * EPS32 * scale
        plg = L.is_plg
        if plg.any():
            tol[plg] = 32 * EPS32 * max(1.0, S.info["cond_A22"][l]) * scale.max()
        worst = float(np.max(np.abs(got - want) / tol))
        print("level %d FP32 sweep: max |diff| / bound = %.3f" % (l, worst))
        assert worst <= 1.0
        if l + 1 < len(H.levels):
            C = H.levels[l + 1]
            want = H.R[l] @ (b - L.A @ u)
            bc = dev32(C, np.zeros(C.n))
            S.restrict(l, dev32(L, b), dev32(L, u), bc)
            au = H.R[l] @ (np.abs(b) + abs(L.A) @ np.abs(u))
            assert np.all(np.abs(back(C, bc) - want) <= 32 * EPS32 * au)
            ec = f32(rng.standard_normal(C.n))
            want = u + H.P[l] @ ec
            ud = dev32(L, u)
            S.prolong(l, dev32(C, ec), ud)
            assert np.all(np.abs(back(L, ud) - want) <= EPS32 * (np.abs(u) + np.abs(H.P[l] @ ec)))


@pytest.mark.parametrize("name", ["disk64", "three_disks128", "star128"])
def test_cond_a22_estimate(name):
    """mg_info.cond_A22 (Hager's estimate of the 1-norm condition number)
    against the oracle's exact value from a dense inverse: a lower bound,
    and within a factor 3 of it."""
    P, H = oracle(name)
    S = product(name, "split_a")
    for l, L in enumerate(H.levels):
        A22 = L.blocks()[3].toarray()
        if A22.shape[0] == 0:
            assert S.info["cond_A22"][l] == 0.0
            continue
        exact = np.linalg.norm(A22, 1) * np.linalg.norm(np.linalg.inv(A22), 1)
        est = S.info["cond_A22"][l]
        print("level %d: cond_1(A22) %.4e, estimate %.4e" % (l, exact, est))
        assert exact / 3 <= est <= exact * (1 + 1e-8)
