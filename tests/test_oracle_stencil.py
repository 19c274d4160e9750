"""Pins of the oracle's ghost and stencil formulas against exact polynomial
reproduction (Section 4.1): checked in exact rational arithmetic, independent
of the tables being tested."""
from fractions import Fraction as Fr

import pytest

from oracle.stencil import (D1, D2, GHOST_DIRICHLET, GHOST_NEUMANN, FACE_EXTRAP,
                            corner_ghost_weights, face_ghost_weights)


def cell_avg_monomial(p, k):
    """Average of x^p over the cell [k, k+1] (h = 1), exactly."""
    return Fr((k + 1) ** (p + 1) - k ** (p + 1), p + 1)


@pytest.mark.parametrize("which", [1, 2])
@pytest.mark.parametrize("p", range(5))
def test_dirichlet_ghost_exact_degree4(which, p):
    # interior cells i-3..i occupy [-4,0]; the face is x = 0; ghost `which`
    # occupies [which-1, which]
    cf = GHOST_DIRICHLET[which - 1]
    interior = [cell_avg_monomial(p, -1 - m) for m in range(4)]      # cells i, i-1, i-2, i-3
    face = Fr(0 ** p) if p else Fr(1)
    val = (sum(Fr(c) * v for c, v in zip(cf[:4], interior)) + cf[4] * face) / cf[5]
    assert val == cell_avg_monomial(p, which - 1)


@pytest.mark.parametrize("which", [1, 2])
@pytest.mark.parametrize("p", range(5))
def test_neumann_ghost_exact_degree4(which, p):
    cf = GHOST_NEUMANN[which - 1]
    interior = [cell_avg_monomial(p, -1 - m) for m in range(4)]
    dudn = Fr(1) if p == 1 else Fr(0)          # d/dx x^p at x = 0 (outward normal +x)
    val = (sum(Fr(c) * v for c, v in zip(cf[:4], interior)) + cf[4] * dudn) / cf[5]
    assert val == cell_avg_monomial(p, which - 1)


def test_printed_face_weight_would_fail():
    # the second Dirichlet ghost with the printed face weight 75 does not even
    # reproduce constants: (27 - 145 + 335 - 505 + 75) / 12 != 1
    cf = GHOST_DIRICHLET[1]
    assert Fr(sum(cf[:4]) + 75, 12) != 1
    assert Fr(sum(cf[:4]) + cf[4], 12) == 1


@pytest.mark.parametrize("p", range(6))
def test_second_derivative_exact_degree5(p):
    # <d2 x^p/dx2> over cell [0,1] from cell averages of cells -2..2
    approx = sum(D2[k] * cell_avg_monomial(p, m) for k, m in enumerate(range(-2, 3)))
    exact = Fr(0) if p < 2 else p * cell_avg_monomial(p - 2, 0) * (p - 1)
    assert approx == exact


@pytest.mark.parametrize("p", range(5))
def test_first_derivative_exact_degree4(p):
    approx = sum(D1[k] * cell_avg_monomial(p, m) for k, m in enumerate(range(-2, 3)))
    exact = Fr(0) if p < 1 else p * cell_avg_monomial(p - 1, 0)
    assert approx == exact


def test_second_derivative_not_exact_degree6():
    approx = sum(D2[k] * cell_avg_monomial(6, m) for k, m in enumerate(range(-2, 3)))
    assert approx != 30 * cell_avg_monomial(4, 0)


BCS = {"D": ("D", 1.0, 0.0), "N": ("N", 0.0, 1.0), "R": ("R", 1.0, 0.5), "R2": ("R", 0.3, 2.0)}


@pytest.mark.parametrize("m,k", [(1, 1), (1, 2), (2, 1), (2, 2)])
@pytest.mark.parametrize("bcx,bcy", [("D", "D"), ("D", "N"), ("N", "N"), ("R", "D"), ("N", "R2"), ("R", "R2")])
def test_corner_ghost_exact_bicubic(m, k, bcx, bcy):
    """A corner ghost reproduces cell averages of x^p y^q for p, q <= 3 given
    exact face data (corner at the origin, interior in x > 0, y > 0, the
    ghost occupies [-m, -m+1] x [-k, -k+1]; h = 1)."""
    wu, wgy, wgx = corner_ghost_weights(BCS[bcx], BCS[bcy], m, k, 1.0)
    ax1, ax2 = BCS[bcx][1], BCS[bcx][2]
    ay1, ay2 = BCS[bcy][1], BCS[bcy][2]
    for p in range(4):
        for q in range(4 - p):
            avg = lambda cx, cy: float(cell_avg_monomial(p, cx) * cell_avg_monomial(q, cy))

            # face data alpha1 u + alpha2 du/dn (Dirichlet (1, 0), Neumann
            # (0, 1)): the y-face (y = 0, outward normal -y) at column P,
            # the x-face (x = 0, outward normal -x) at row Q
            def gy(P):
                a = float(cell_avg_monomial(p, P))
                return ay1 * a * (1.0 if q == 0 else 0.0) - ay2 * a * (1.0 if q == 1 else 0.0)

            def gx(Q):
                a = float(cell_avg_monomial(q, Q))
                return ax1 * a * (1.0 if p == 0 else 0.0) - ax2 * a * (1.0 if p == 1 else 0.0)
            val = sum(wu[a][b] * avg(a, b) for a in range(4) for b in range(4))
            val += sum(wgy[a] * gy(a) for a in range(4)) + sum(wgx[b] * gx(b) for b in range(4))
            assert val == pytest.approx(avg(-m, -k), abs=1e-9)


@pytest.mark.parametrize("which", [1, 2])
@pytest.mark.parametrize("alpha1,alpha2,h", [(1.0, 0.5, 1.0 / 64), (0.3, 2.0, 1.0 / 8), (2.0, 0.01, 0.5)])
def test_robin_ghost_exact_degree4(which, alpha1, alpha2, h):
    """The Robin ghost (reading of Sec. 4.1: the degree-4 reconstruction with
    alpha1 u + alpha2 du/dn as the face condition) reproduces the ghost
    average of every monomial of degree <= 4 in the physical normal
    coordinate X = h x (face at X = 0, outward normal +X)."""
    w = face_ghost_weights("R", alpha1, alpha2, h, which)
    for p in range(5):
        # X^p = h^p x^p: cell averages scale by h^p, d/dX at 0 is 1 for p = 1
        interior = [h ** p * float(cell_avg_monomial(p, -1 - m)) for m in range(4)]
        g = alpha1 * (1.0 if p == 0 else 0.0) + alpha2 * (1.0 if p == 1 else 0.0)
        val = sum(c * v for c, v in zip(w[:4], interior)) + w[4] * g
        assert val == pytest.approx(h ** p * float(cell_avg_monomial(p, which - 1)), abs=1e-11 * max(1.0, h ** p))


@pytest.mark.parametrize("which", [1, 2])
def test_robin_ghost_reduces_to_the_printed_formulas(which):
    """alpha2 = 0 gives the Dirichlet ghost, alpha1 = 0 the Neumann ghost
    (whose face weight multiplies h g)."""
    h = 1.0 / 32
    d = GHOST_DIRICHLET[which - 1]
    n = GHOST_NEUMANN[which - 1]
    wd = face_ghost_weights("R", 1.0, 0.0, h, which)
    wn = face_ghost_weights("R", 0.0, 1.0, h, which)
    assert wd == pytest.approx([v / d[5] for v in d[:5]], abs=1e-12)
    assert wn[:4] == pytest.approx([v / n[5] for v in n[:4]], abs=1e-12)
    assert wn[4] == pytest.approx(n[4] / n[5] * h, abs=1e-14)


def test_face_extrapolation_cubic():
    for m in (1, 2):
        for p in range(4):
            val = sum(FACE_EXTRAP[m - 1][a] * a ** p for a in range(4))
            assert val == (-m) ** p
