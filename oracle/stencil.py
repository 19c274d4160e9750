"""Ghost filling and the symmetric fourth-order FV formulas (Section 4.1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Ghost cells (Section 4.1): for an extendable face at the high end of cells
i-3, i-2, i-1, i (all regular), two ghost cells i+1, i+2 receive cell averages
extrapolated from those four cells and the face datum.  The coefficients are
stored as (c_i, c_{i-1}, c_{i-2}, c_{i-3}, c_face, denominator); the face
datum enters as g for Dirichlet and as h*g (g the outward normal derivative)
for Neumann.

Reading of a garbled coefficient: the printed face weight of the second
Dirichlet ghost cannot be right, because the weights must sum to the
denominator for the formula to reproduce constants; the value that makes the
formula exact for all polynomials of degree <= 4 is 300/12, and that is the
value used here.

Symmetric FV formulas, eqs. (4.7a,b):
  <d phi/dx_d>_i    = (phi_{i-2} - 8 phi_{i-1} + 8 phi_{i+1} - phi_{i+2}) / (12 h)
  <d2 phi/dx_d^2>_i = (-phi_{i-2} + 16 phi_{i-1} - 30 phi_i + 16 phi_{i+1} - phi_{i+2}) / (12 h^2)
and the cross derivative applies the first formula in x and then in y.
"""
from fractions import Fraction as Fr

import numpy as np

# (c_i, c_{i-1}, c_{i-2}, c_{i-3}, c_face, denominator) for ghosts i+1 and i+2
GHOST_DIRICHLET = ((-77, 43, -17, 3, 60, 12), (-505, 335, -145, 27, 300, 12))
GHOST_NEUMANN = ((5, 9, -5, 1, 12, 10), (-15, 29, -15, 3, 12, 2))

# Corner ghost cells (outside the box in both directions, reached only by the
# cross-derivative stencil near the box corners).  The paper defines ghost
# cells for faces only.  Here a corner ghost is the face-ghost formula of one
# face applied to the ghost cells of the other face, averaged over the two
# orders.  The only missing datum, the face average of the other face one or
# two cells beyond the corner, is the cubic extrapolation of that face's data
# along the face (weights below on the data 0..3 cells from the corner).
# Other choices tried: treating the cells that reach the corner as PLG cells
# and extrapolating the interior polynomially both make the two-grid operator
# converge far worse or diverge, while this choice reproduces the two-grid
# rates of the b = 0 case.
FACE_EXTRAP = ((4, -6, 4, -1), (10, -20, 15, -4))

D1 = (Fr(1, 12), Fr(-8, 12), Fr(0), Fr(8, 12), Fr(-1, 12))          # offsets -2..2, times 1/h
D2 = (Fr(-1, 12), Fr(16, 12), Fr(-30, 12), Fr(16, 12), Fr(-1, 12))  # offsets -2..2, times 1/h^2


def ghost_table(bc):
    if bc == "D":
        return GHOST_DIRICHLET
    if bc == "N":
        return GHOST_NEUMANN
    raise ValueError("ghost cells are defined for Dirichlet and Neumann faces only")


def ghost_weights(bc, which):
    """Float weights (w_i, w_{i-1}, w_{i-2}, w_{i-3}, w_face) of ghost `which`
    (1 or 2).  For Neumann the face weight multiplies h * <du/dn>."""
    c = ghost_table(bc)[which - 1]
    return tuple(float(Fr(v, c[5])) for v in c[:5])


def face_ghost_weights(bc, alpha1, alpha2, h, which):
    """(w_i, w_{i-1}, w_{i-2}, w_{i-3}, w_g) of ghost `which` (1 or 2) with the
    face datum g entering as given: g = u on a Dirichlet face, g = du/dn on a
    Neumann face (the tables above, face weight times h), and
    g = alpha1 u + alpha2 du/dn on a Robin face.

    Reading for Robin (Section 4.1 gives Dirichlet, Neumann and periodic
    ghosts only): the same construction as the other two, i.e. the polynomial
    p of degree 4 in the normal coordinate x (cell widths 1, the face at
    x = 0, the cells i, i-1, i-2, i-3 on [-1, 0], ..., [-4, -3], the outward
    normal along +x) whose averages over the four cells are u_i .. u_{i-3} and
    with alpha1 p(0) + alpha2 p'(0) / h = g; the ghost is p's average over
    [which - 1, which]."""
    if bc in ("D", "N"):
        w = ghost_weights(bc, which)
        return w[:4] + (w[4] * (h if bc == "N" else 1.0),)

    def avg(a, k):                      # average of x^k over [a, a + 1]
        return ((a + 1.0) ** (k + 1) - a ** (k + 1)) / (k + 1)

    M = np.zeros((5, 5))
    for m in range(4):                  # cell i - m on [-(m + 1), -m]
        M[m] = [avg(-(m + 1.0), k) for k in range(5)]
    M[4, 0], M[4, 1] = alpha1, alpha2 / h
    e = np.array([avg(which - 1.0, k) for k in range(5)])
    return tuple(float(v) for v in np.linalg.solve(M.T, e))


def operator_terms(a, b, c, h):
    """The SFV stencil of L = a d_xx + b d_xy + c d_yy as a list of
    ((m1, m2), weight) over offsets in [-2, 2]^2 (eq. (4.7) and the mixed term)."""
    terms = {}
    for k, m in enumerate(range(-2, 3)):
        terms[(m, 0)] = terms.get((m, 0), 0.0) + a * float(D2[k]) / (h * h)
        terms[(0, m)] = terms.get((0, m), 0.0) + c * float(D2[k]) / (h * h)
    if b != 0.0:
        for k1, m1 in enumerate(range(-2, 3)):
            for k2, m2 in enumerate(range(-2, 3)):
                w = float(D1[k1] * D1[k2])
                if w != 0.0:
                    terms[(m1, m2)] = terms.get((m1, m2), 0.0) + b * w / (h * h)
    return sorted(terms.items())


def corner_ghost_weights(bcx, bcy, m, k, h):
    """Weights of the corner ghost m cells beyond the x-face and k cells beyond
    the y-face; bcx, bcy: (bc, alpha1, alpha2) of the two faces.  Returns
    (wu, wgy, wgx): wu[p][q] on the interior cell p steps inward in x and q
    steps inward in y; wgy[p] on the y-face datum at the column p steps
    inward; wgx[q] on the x-face datum at the row q steps inward.  Face data
    enter as in ``face_ghost_weights``."""
    gx = face_ghost_weights(bcx[0], bcx[1], bcx[2], h, m)
    gy = face_ghost_weights(bcy[0], bcy[1], bcy[2], h, k)
    ex, ey = FACE_EXTRAP[m - 1], FACE_EXTRAP[k - 1]
    wu = [[gx[p] * gy[q] for q in range(4)] for p in range(4)]
    wgy = [0.5 * gy[4] * (gx[p] + ex[p]) for p in range(4)]
    wgx = [0.5 * gx[4] * (gy[q] + ey[q]) for q in range(4)]
    return wu, wgy, wgx
