"""The linear system A u = f - N g of one level (Section 4).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Steps, in the paper's order:
  * extendable faces and cells, ghost cells           (Section 4.1)
  * SFV / PLG classification                          (Definition 4.1, eq. (4.6))
  * SFV rows from eq. (4.7) with ghosts eliminated    (Section 4.1)
  * a poised lattice S_PLG(i) for every PLG cell      (Definitions 4.2-4.3)
  * the stencil X(i) (eq. (4.10)), the sample matrix M (eq. (4.13)), the
    weights W (eq. (4.17)) and the minimum-norm coefficients
    beta = W M^T (M W M^T)^{-1} phibar (eq. (4.16), Lemma 4.4)
  * the global system and its block form (eqs. (4.19)-(4.21))

Readings of points the paper leaves open:
  * the outer boundary is the grid box; every box face must be extendable on
    every level (otherwise that level is rejected);
  * positions of S_i outside the box in both coordinates (reached only by
    the cross-derivative stencil near the box corners) are corner ghost cells,
    filled by composing the two face-ghost formulas (see ``stencil``);
    treating the cells that reach them as PLG cells instead makes the block
    smoother diverge (spectral radius above 1 on the unit square);
  * lattice selection (the cited PLG algorithm is not reproduced): K is the
    set of active cells in the 7x7 index box centred at i (9x9 if needed);
    a nearest-first greedy with an exact rank test is run under each of the
    8 grid symmetries (see ``candidate_lattices``); each candidate is fitted
    for the actual cell, and the one whose row is the most diagonally
    dominant with a negative own coefficient is kept (``Level._lattice``).
    Ranking candidates by the weighted norm of a full-cell fit instead
    leaves rows with a positive own coefficient near curved Neumann and
    Robin boundaries and with a strong cross term, which make the two-grid
    correction diverge; widening the candidates (shifted centres, 9x9 boxes)
    improves the worst rows further but slows the V- and FMG cycles down;
  * the basis centre p is the centre of the grid cell of i;
  * the minimum-W^{-1}-norm solution is computed as beta = W^{1/2} gamma with
    gamma the minimum-2-norm solution of (M W^{1/2}) gamma = phibar, which is
    the same vector as eq. (4.16) without forming M W M^T.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .geometry import (MONOS, MONO_INDEX, CutGrid, GeometryError, _GL, full_cell_moments, seg_deriv,
                       seg_normal, seg_point, shift_moments)
from .stencil import corner_ghost_weights, face_ghost_weights, operator_terms

NBASIS = len(MONOS)        # dim Pi_4^2 = 15
W_MIN = 0.5                # eq. (4.17)

SFV, PLG = 1, 2


# ----------------------------------------------------------------------------
# lattices
# ----------------------------------------------------------------------------
def _mono_row(d):
    return [d[0] ** a * d[1] ** b for a, b in MONOS]


class _Echelon:
    """Incremental row echelon form over the integers (fraction-free, exact
    rank test over the rationals)."""

    def __init__(self):
        self.rows = []           # (pivot column, row)

    def try_add(self, v):
        v = list(v)
        for piv, r in self.rows:
            if v[piv] != 0:
                f, g = r[piv], v[piv]
                v = [f * x - g * y for x, y in zip(v, r)]
                # keep the entries small: divide by the gcd
                gg = 0
                for x in v:
                    gg = math.gcd(gg, x)
                if gg > 1:
                    v = [x // gg for x in v]
        for k, x in enumerate(v):
            if x != 0:
                self.rows.append((k, v))
                return True
        return False


def _greedy(cands):
    ech = _Echelon()
    chosen = []
    for d in cands:
        if ech.try_add(_mono_row(d)):
            chosen.append(d)
            if len(chosen) == NBASIS:
                return chosen
    return None


def _angle(d):
    return math.atan2(d[1], d[0]) % (2.0 * math.pi)


_LATTICE_MEMO = {}

# the 8 symmetries of the grid (rotations by 90 degrees and reflections)
_SYMMETRIES = ((1, 0, 0, 1), (0, -1, 1, 0), (-1, 0, 0, -1), (0, 1, -1, 0),
               (1, 0, 0, -1), (0, 1, 1, 0), (-1, 0, 0, 1), (0, -1, -1, 0))


def candidate_lattices(window):
    """window: frozenset of offsets d (|d|_inf <= 4) of the active cells around
    the PLG cell i.  Returns the poised lattices S_PLG(i) the selection chooses
    from (Definitions 4.2-4.3).

    K is the set of active cells in the 7x7 box centred at i (the 9x9 box if
    the 7x7 one holds no poised subset).  For each of the 8 symmetries g of
    the grid, nodes of K are taken nearest-first, ordered by (|d|^2, angle of
    g(d) in [0, 2pi)), whenever they raise the exact rank of the point-sample
    matrix [d^alpha], |alpha| <= 4, until 15 are chosen.  Each lattice starts
    with d = (0, 0).  Distinct lattices are returned in symmetry order."""
    hit = _LATTICE_MEMO.get(window)
    if hit is not None:
        return hit
    out = []
    for half in (3, 4):
        box = [d for d in window if abs(d[0]) <= half and abs(d[1]) <= half]
        if len(box) < NBASIS:
            continue
        for g in _SYMMETRIES:
            order = sorted(box, key=lambda d: (d[0] * d[0] + d[1] * d[1],
                                               _angle((g[0] * d[0] + g[1] * d[1], g[2] * d[0] + g[3] * d[1]))))
            lat = _greedy(order)
            if lat is not None and lat not in out:
                out.append(lat)
        if out:
            break
    if not out:
        raise GeometryError("no poised lattice for a PLG cell")
    _LATTICE_MEMO[window] = out
    return out


def row_dominance(beta):
    """Selection key of a fitted PLG row whose lattice starts at the cell
    itself: sum_{k>0} |beta_k| / (-beta_0) when the cell's own coefficient is
    negative (the sign of the operator's diagonal), else +inf."""
    if beta[0] >= 0.0:
        return math.inf
    return float(np.sum(np.abs(beta[1:]))) / float(-beta[0])


# ----------------------------------------------------------------------------
# one level
# ----------------------------------------------------------------------------
class Level:
    """Cut cells, classification and the assembled system of one grid."""

    def __init__(self, grid, curves, a, b, c, eps, omega=0.5, progress=None, w_min=W_MIN):
        """progress: optional callable(str) told when each stage is done;
        w_min: the smallest weight of eq. (4.17) and the boundary weight."""
        self.grid = grid
        self.w_min = float(w_min)
        self.a, self.b, self.c = float(a), float(b), float(c)
        self.h, self.nx, self.ny = grid.h, grid.nx, grid.ny
        self.curves = curves
        note = progress or (lambda msg: None)
        self.cg = CutGrid(grid, curves, eps)
        note("%dx%d: cut cells" % (grid.nx, grid.ny))
        self._classify()
        self._index()
        note("%dx%d: classification" % (grid.nx, grid.ny))
        self._assemble()
        note("%dx%d: assembly" % (grid.nx, grid.ny))

    # -- Definition 4.1 ---------------------------------------------------------
    def _classify(self):
        nx, ny = self.nx, self.ny
        R = self.cg.regular
        if nx < 4 or ny < 4:
            raise GeometryError("grid too small for ghost cells")
        # a box face is extendable when the 4 cells inward from it are regular
        for j in range(ny):
            if not (R[j, 0:4].all() and R[j, nx - 4:nx].all()):
                raise GeometryError("a box face is not extendable")
        for i in range(nx):
            if not (R[0:4, i].all() and R[ny - 4:ny, i].all()):
                raise GeometryError("a box face is not extendable")
        ok = np.zeros((ny + 4, nx + 4), bool)     # regular cell or ghost cell
        ok[2:ny + 2, 2:nx + 2] = R
        ok[2:ny + 2, 0:2] = True                  # left ghosts (rows inside)
        ok[2:ny + 2, nx + 2:] = True              # right ghosts
        ok[0:2, 2:nx + 2] = True                  # bottom ghosts
        ok[ny + 2:, 2:nx + 2] = True              # top ghosts
        for sl_y in (slice(0, 2), slice(ny + 2, ny + 4)):
            for sl_x in (slice(0, 2), slice(nx + 2, nx + 4)):
                ok[sl_y, sl_x] = True             # corner ghosts
        if self.b == 0.0:
            offs = [(m, 0) for m in range(-2, 3)] + [(0, m) for m in (-2, -1, 1, 2)]
        else:
            offs = [(m1, m2) for m1 in range(-2, 3) for m2 in range(-2, 3)]
        sfv = np.ones((ny, nx), bool)
        for dx, dy in offs:
            sfv &= ok[2 + dy:ny + 2 + dy, 2 + dx:nx + 2 + dx]
        act = self.cg.active
        self.kind = np.zeros((ny, nx), np.int8)
        self.kind[act & sfv] = SFV
        self.kind[act & ~sfv] = PLG

    def _index(self):
        nx, ny = self.nx, self.ny
        act = self.cg.active
        self.idx = -np.ones((ny, nx), np.int64)
        jj, ii = np.nonzero(act)                  # row-major order
        self.n = len(ii)
        self.idx[jj, ii] = np.arange(self.n)
        self.cells_i, self.cells_j = ii, jj
        self.is_plg = self.kind[jj, ii] == PLG
        # boundary data layout: box faces, then irregular PLG cells (row-major)
        self.n_face = 2 * nx + 2 * ny
        irr = [(i, j) for j, i in zip(jj, ii) if not self.cg.regular[j, i]]
        self.irregular = irr
        self.g_irr = {cell: self.n_face + k for k, cell in enumerate(irr)}
        self.n_g = self.n_face + len(irr)

    def face_index(self, side, k):
        """g index of box face k on side 0=bottom, 1=right, 2=top, 3=left."""
        nx, ny = self.nx, self.ny
        return (k, 2 * nx + ny + k, nx + k, 2 * nx + k)[side]

    # -- eqs. (4.7), (4.10)-(4.21) -----------------------------------------------
    def _assemble(self):
        nx, ny, h = self.nx, self.ny, self.h
        terms = operator_terms(self.a, self.b, self.c, h)
        rows, cols, vals = [], [], []
        nrows, ncols, nvals = [], [], []
        sj, si = np.nonzero(self.kind == SFV)
        srow = self.idx[sj, si]
        box_bc = self.cg.box_bc
        # periodic box sides (Sec. 4.1): a position beyond the box in a
        # periodic direction is the cell one period away; what is still
        # outside afterwards takes the ghost formulas of the other sides
        per_x, per_y = box_bc[1][0] == "P", box_bc[0][0] == "P"
        for (m1, m2), w in terms:
            qi, qj = si + m1, sj + m2
            if per_x:
                qi = qi % nx
            if per_y:
                qj = qj % ny
            inside = (qi >= 0) & (qi < nx) & (qj >= 0) & (qj < ny)
            rows.append(srow[inside]); cols.append(self.idx[qj[inside], qi[inside]])
            vals.append(np.full(inside.sum(), w))
            # corner ghosts: outside in both coordinates
            corner = ((qi < 0) | (qi >= nx)) & ((qj < 0) | (qj >= ny))
            for k in np.nonzero(corner)[0]:
                r, cx, cy = srow[k], int(qi[k]), int(qj[k])
                xside, m = (3, -cx) if cx < 0 else (1, cx - nx + 1)
                yside, kk = (0, -cy) if cy < 0 else (2, cy - ny + 1)
                wu, wgy, wgx = corner_ghost_weights(box_bc[xside], box_bc[yside], m, kk, h)
                colx = lambda p: p if xside == 3 else nx - 1 - p
                rowy = lambda q: q if yside == 0 else ny - 1 - q
                for p in range(4):
                    for q in range(4):
                        rows.append(np.array([r])); cols.append(np.array([self.idx[rowy(q), colx(p)]]))
                        vals.append(np.array([w * wu[p][q]]))
                    nrows.append(np.array([r])); ncols.append(np.array([self.face_index(yside, colx(p))]))
                    nvals.append(np.array([w * wgy[p]]))
                    nrows.append(np.array([r])); ncols.append(np.array([self.face_index(xside, rowy(p))]))
                    nvals.append(np.array([w * wgx[p]]))
            # face ghosts: outside in exactly one coordinate
            for side in range(4):
                if side == 0:
                    sel = (qj < 0) & (qi >= 0) & (qi < nx); depth = -qj; along = qi
                elif side == 2:
                    sel = (qj >= ny) & (qi >= 0) & (qi < nx); depth = qj - ny + 1; along = qi
                elif side == 3:
                    sel = (qi < 0) & (qj >= 0) & (qj < ny); depth = -qi; along = qj
                else:
                    sel = (qi >= nx) & (qj >= 0) & (qj < ny); depth = qi - nx + 1; along = qj
                if not sel.any():
                    continue
                bc = box_bc[side]
                for which in (1, 2):
                    s2 = sel & (depth == which)
                    if not s2.any():
                        continue
                    gw = face_ghost_weights(bc[0], bc[1], bc[2], h, which)
                    al = along[s2]
                    r = srow[s2]
                    for k in range(4):          # interior cell k steps inward
                        if side == 0:
                            ci, cj = al, np.full(al.shape, k)
                        elif side == 2:
                            ci, cj = al, np.full(al.shape, ny - 1 - k)
                        elif side == 3:
                            ci, cj = np.full(al.shape, k), al
                        else:
                            ci, cj = np.full(al.shape, nx - 1 - k), al
                        rows.append(r); cols.append(self.idx[cj, ci])
                        vals.append(np.full(r.shape, w * gw[k]))
                    fw = gw[4]
                    nrows.append(r)
                    ncols.append(np.array([self.face_index(side, int(k)) for k in al], np.int64))
                    nvals.append(np.full(r.shape, w * fw))
        # PLG rows
        self.lattice = {}
        self.beta = {}
        pj, pi_ = np.nonzero(self.kind == PLG)
        for i, j in zip(pi_, pj):
            i, j = int(i), int(j)
            lat = self._lattice(i, j)
            beta, bb = self._fit(i, j, lat)
            self.lattice[(i, j)] = lat
            self.beta[(i, j)] = (beta, bb)
            r = self.idx[j, i]
            rows.append(np.full(len(lat), r))
            cols.append(np.array([self.idx[j + d[1], i + d[0]] for d in lat]))
            vals.append(beta)
            if bb is not None:
                nrows.append(np.array([r])); ncols.append(np.array([self.g_irr[(i, j)]]))
                nvals.append(np.array([bb]))
        self.A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                               shape=(self.n, self.n))
        self.A.sum_duplicates()
        if nrows:
            self.N = sp.csr_matrix((np.concatenate(nvals), (np.concatenate(nrows), np.concatenate(ncols))),
                                   shape=(self.n, self.n_g))
        else:
            self.N = sp.csr_matrix((self.n, self.n_g))
        self.N.sum_duplicates()

    def _lattice(self, i, j):
        """S_PLG(i): of the candidate lattices, the one whose fitted row (for
        this cell, its neighbours and B_i) is the most diagonally dominant
        (smallest row_dominance); a key within a relative 1e-9 of the best so
        far keeps the earlier candidate; with no negative diagonal among the
        candidates, the first candidate."""
        win = frozenset((dx, dy) for dx in range(-4, 5) for dy in range(-4, 5)
                        if self.cg.is_active(i + dx, j + dy))
        cands = candidate_lattices(win)
        best, bestv = cands[0], math.inf
        for lat in cands:
            beta, _ = self._fit(i, j, lat)
            v = row_dominance(beta)
            if v < bestv * (1.0 - 1e-9):
                best, bestv = lat, v
        return best

    def _avg_monomials(self, cell, d):
        """<((x - p)/h)^alpha>_cell for p the centre of grid cell cell - d."""
        mom = self.cg.cell_moments(cell)
        return shift_moments(mom, d[0], d[1]) / mom[0]

    def _lphi(self, i, j):
        """phibar_alpha = <L phi_alpha>_i (eq. (4.13))."""
        mom = self.cg.cell_moments((i, j))
        avg = mom / mom[0]
        out = np.zeros(NBASIS)
        h2 = self.h * self.h
        for k, (p, q) in enumerate(MONOS):
            s = 0.0
            if p >= 2:
                s += self.a * p * (p - 1) * avg[MONO_INDEX[(p - 2, q)]]
            if p >= 1 and q >= 1:
                s += self.b * p * q * avg[MONO_INDEX[(p - 1, q - 1)]]
            if q >= 2:
                s += self.c * q * (q - 1) * avg[MONO_INDEX[(p, q - 2)]]
            out[k] = s / h2
        return out

    def boundary_average_of_basis(self, i, j):
        """<<N phi_alpha>>_{B_i} for all alpha (the last column of eq. (4.13))."""
        h = self.h
        xc, yc = self.grid.x0 + (i + 0.5) * h, self.grid.y0 + (j + 0.5) * h
        s, w = _GL[16]
        tot = np.zeros(NBASIS)
        length = 0.0
        for ci, si, ta, tb in self.cg.cells[(i, j)]["bpieces"]:
            seg = self.curves[ci][si]
            t = 0.5 * (tb - ta) * s + 0.5 * (ta + tb)
            x, y = seg_point(seg, t)
            dx, dy = seg_deriv(seg, t)
            ds = 0.5 * (tb - ta) * w * np.hypot(dx, dy)
            nxv, nyv = seg_normal(seg, t)
            X, Y = (x - xc) / h, (y - yc) / h
            for k, (p, q) in enumerate(MONOS):
                phi = X ** p * Y ** q
                gx = p * X ** (p - 1) * Y ** q / h if p >= 1 else 0.0 * X
                gy = q * X ** p * Y ** (q - 1) / h if q >= 1 else 0.0 * X
                dn = gx * nxv + gy * nyv
                if seg.bc == "D":
                    val = phi
                elif seg.bc == "N":
                    val = dn
                else:
                    val = seg.alpha1 * phi + seg.alpha2 * dn
                tot[k] += np.sum(ds * val)
            length += float(np.sum(ds))
        return tot / length

    def _fit(self, i, j, lat):
        """Minimum-norm coefficients of eqs. (4.14)-(4.18)."""
        M = np.empty((NBASIS, len(lat)))
        for k, d in enumerate(lat):
            M[:, k] = self._avg_monomials((i + d[0], j + d[1]), d)
        wk = np.array([max(math.hypot(d[0], d[1]), self.w_min) for d in lat])
        phibar = self._lphi(i, j)
        if self.cg.regular[j, i]:
            return np.linalg.solve(M, phibar), None
        M = np.hstack([M, self.boundary_average_of_basis(i, j)[:, None]])
        wk = np.append(wk, self.w_min)
        sq = 1.0 / np.sqrt(wk)                  # W^{1/2}, W = diag(1/w_k)
        gamma = np.linalg.lstsq(M * sq[None, :], phibar, rcond=None)[0]
        beta = sq * gamma
        return beta[:-1], float(beta[-1])

    # -- block form (eq. (4.21)) -------------------------------------------------
    def blocks(self):
        p = self.is_plg
        s = ~p
        A = self.A.tocsr()
        return (A[s][:, s], A[s][:, p], A[p][:, s], A[p][:, p])

    def to_grid(self, v):
        out = np.zeros((self.ny, self.nx))
        out[self.cells_j, self.cells_i] = v
        return out

    def from_grid(self, g):
        return np.asarray(g)[self.cells_j, self.cells_i]
