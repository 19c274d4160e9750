"""Block smoother, transfers, V-cycle and the outer iteration (Section 5).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

  * block smoother, Definition 5.6: weighted Jacobi on the SFV unknowns with
    the old PLG unknowns (eq. (5.5)), then an exact solve of the PLG block
    A22 u2 = b2 - A21 u1 (eq. (5.6)); omega = 1/2.  The exact solve uses a
    sparse LU of A22 (any exact solve gives the same u2; the banded LU of
    Definition 5.3 is one way to obtain it);
  * level hierarchy, eq. (5.7): every level is its own run of Algorithm 1
    and its own discretisation;
  * restriction eq. (5.8) and piecewise-constant interpolation eq. (5.9);
  * V-cycle, Algorithm 3, with a direct bottom solve;
  * outer iteration: V-cycles until ||b - A u||_inf <= tol ||b||_inf.

Readings of points the paper leaves open:
  * D11 in eq. (5.5) is the centre weight -5(a+c)/(2h^2) of the symmetric FV
    formulas for every SFV row, including rows whose stencil reaches ghost
    cells (the ghosts are filled from the current iterate and treated as
    given); with this reading the two-grid spectral radii of Table 1 on the
    unit square are reproduced to every printed digit;
  * a fine cell whose parent index floor(i/2) is no cut cell of the coarse
    level (it was merged away) is mapped to the coarse cell that absorbed it;
  * coarse levels see homogeneous boundary data (the residual equation);
  * levels: coarsen while the coarser grid is valid (every box face
    extendable, Algorithm 1 succeeds, every PLG cell has a lattice) and has
    at least 16 cells per side, unless the number of levels is given.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretize import Level
from .geometry import GeometryError


class _Grid:
    def __init__(self, x0, y0, h, nx, ny):
        self.x0, self.y0, self.h, self.nx, self.ny = x0, y0, h, nx, ny


class Hierarchy:
    def __init__(self, grid, curves, a, b, c, eps, n_levels=0, omega=0.5, nu=(3, 3), min_cells=16,
                 progress=None, w_min=0.5, colouring=False, block=(64, 16)):
        self.omega = float(omega)
        self.colouring = bool(colouring)
        self.block = block
        self.nu1, self.nu2 = nu
        self.levels = [Level(grid, curves, a, b, c, eps, progress=progress, w_min=w_min)]
        while n_levels == 0 or len(self.levels) < n_levels:
            g = self.levels[-1].grid
            if g.nx % 2 or g.ny % 2 or g.nx // 2 < min_cells or g.ny // 2 < min_cells:
                if n_levels:
                    raise GeometryError("cannot build the requested number of levels")
                break
            cg = _Grid(g.x0, g.y0, 2 * g.h, g.nx // 2, g.ny // 2)
            try:
                self.levels.append(Level(cg, curves, a, b, c, eps, progress=progress, w_min=w_min))
            except GeometryError:
                if n_levels:
                    raise
                break
        self.R = [self._restriction(l) for l in range(len(self.levels) - 1)]
        self.P = [4.0 * R.T.tocsr() for R in self.R]
        self._smoother_setup()
        self.bottom = spla.splu(self.levels[-1].A.tocsc())

    def _restriction(self, l):
        """I_h^{2h} of eq. (5.8) as a sparse matrix (coarse x fine)."""
        fine, coarse = self.levels[l], self.levels[l + 1]
        ci, cj = fine.cells_i // 2, fine.cells_j // 2
        parent = coarse.idx[cj, ci].copy()
        for k in np.nonzero(parent < 0)[0]:
            cell = (int(ci[k]), int(cj[k]))
            own = coarse.cg.owner.get(cell)
            if own is None:
                raise GeometryError("fine cell without a coarse parent")
            parent[k] = coarse.idx[own[1], own[0]]
        return sp.csr_matrix((np.full(fine.n, 0.25), (parent, np.arange(fine.n))),
                             shape=(coarse.n, fine.n))

    def _smoother_setup(self):
        self.sm = []
        for L in self.levels:
            A11, A12, A21, A22 = L.blocks()
            # D11: the centre weight of the symmetric FV operator, -5(a+c)/(2h^2),
            # for every SFV row (ghost values count as given during a sweep).
            # This reading reproduces Table 1 to all printed digits; using the
            # diagonal after ghost elimination does not.
            d11 = np.full(A11.shape[0], -2.5 * (L.a + L.c) / (L.h * L.h))
            lu22 = spla.splu(A22.tocsc()) if A22.shape[0] else None
            # colours of the SFV cells for the multicolour variant: (i + j)
            # mod 3 for the plus-shaped stencil (b = 0), (i + 3 j) mod 9 for
            # the 5 x 5 box (b != 0); no two cells of one colour are within
            # each other's stencil
            s_cells = ~L.is_plg
            ci, cj = L.cells_i[s_cells], L.cells_j[s_cells]
            colour = (ci + cj) % 3 if L.b == 0.0 else (ci + 3 * cj) % 9
            a_in = self._block_part(L, ci, cj) if self.colouring else None
            self.sm.append((A11, A12, A21, A22, d11, lu22, s_cells, L.is_plg, colour, a_in))

    def _block_part(self, L, ci, cj):
        """The part of A11 that the multicolour variant takes from the current
        values: the stencil weights of eq. (4.7) (and the mixed term) between
        SFV cells of the same block of self.block cells; everything else
        (other blocks, ghost values) comes from the sweep's starting values."""
        from .stencil import operator_terms
        bx, by = self.block
        pos = -np.ones((L.ny, L.nx), dtype=np.int64)
        pos[cj, ci] = np.arange(len(ci))
        rows, cols, vals = [], [], []
        for (m1, m2), w in operator_terms(L.a, L.b, L.c, L.h):
            ni, nj = ci + m1, cj + m2
            ok = (ni >= 0) & (ni < L.nx) & (nj >= 0) & (nj < L.ny)
            ok &= (ni // bx == ci // bx) & (nj // by == cj // by)
            k = np.nonzero(ok)[0]
            tgt = pos[nj[k], ni[k]]
            keep = tgt >= 0
            rows.append(k[keep]); cols.append(tgt[keep]); vals.append(np.full(int(keep.sum()), w))
        n = len(ci)
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))

    # -- Definition 5.6 ---------------------------------------------------------
    def smooth(self, l, u, b):
        A11, A12, A21, A22, d11, lu22, s, p, colour, a_in = self.sm[l]
        u = u.copy()
        u1, u2 = u[s], u[p]
        if self.colouring:
            # multicolour variant (an extension): the update of eq. (5.5)
            # applied colour by colour; within a block each colour sees the
            # values the previous colours left, across blocks and through
            # ghost cells the values at the start of the sweep
            r_rest = b[s] - (A11 - a_in) @ u1 - A12 @ u2
            for k in range(int(colour.max()) + 1 if len(colour) else 0):
                sel = colour == k
                r = r_rest - a_in @ u1
                u1[sel] = u1[sel] + self.omega * r[sel] / d11[sel]
        else:
            u1 = u1 + self.omega * (b[s] - A11 @ u1 - A12 @ u2) / d11    # eq. (5.5)
        if lu22 is not None:
            u2 = lu22.solve(b[p] - A21 @ u1)                                # eq. (5.6)
        u[s], u[p] = u1, u2
        return u

    # -- Algorithm 3 -----------------------------------------------------------
    def vcycle(self, l, u, b):
        L = self.levels[l]
        if l == len(self.levels) - 1:
            return self.bottom.solve(b)
        for _ in range(self.nu1):
            u = self.smooth(l, u, b)
        r2 = self.R[l] @ (b - L.A @ u)
        e2 = self.vcycle(l + 1, np.zeros(self.levels[l + 1].n), r2)
        u = u + self.P[l] @ e2
        for _ in range(self.nu2):
            u = self.smooth(l, u, b)
        return u

    # -- Algorithm 4 -----------------------------------------------------------
    def fmg(self, l, r):
        """FMG cycle on the residual equation A^h e = r^h; returns e."""
        if l == len(self.levels) - 1:
            return self.bottom.solve(r)
        e2 = self.fmg(l + 1, self.R[l] @ r)
        e = self.P[l] @ e2
        return self.vcycle(l, e, r)

    def solve(self, b, u0=None, tol=1e-10, max_iters=100, history=None, cycle="V"):
        """Outer iteration with V-cycles (u <- Vcycle(u, b)) or FMG cycles on
        the residual equation (u <- u + FMG(b - A u), Section 5.4); returns
        (u, iterations, relative residual)."""
        A = self.levels[0].A
        u = np.zeros_like(b) if u0 is None else u0.copy()
        bn = np.abs(b).max()
        rel = np.abs(b - A @ u).max() / bn
        it = 0
        while rel > tol and it < max_iters:
            if cycle == "V":
                u = self.vcycle(0, u, b)
            else:
                u = u + self.fmg(0, b - A @ u)
            it += 1
            rel = np.abs(b - A @ u).max() / bn
            if history is not None:
                history.append((u.copy(), rel))
        return u, it, rel

    # -- eq. (5.10) -----------------------------------------------------------
    def two_grid_operator(self, nu1, nu2):
        """TG = T^nu2 [I - P (A^{2h})^{-1} R A^h] T^nu1 as a LinearOperator on
        level 0, with the coarse solve exact (parity unpinned for domains with
        PLG cells; pinned on the unit square by Table 1)."""
        A = self.levels[0].A
        lu_c = spla.splu(self.levels[1].A.tocsc())
        R, P = self.R[0], self.P[0]
        zero = np.zeros(A.shape[0])

        def T(e):
            return self.smooth(0, e, zero)

        def mv(e):
            e = np.asarray(e).ravel()
            for _ in range(nu1):
                e = T(e)
            e = e - P @ lu_c.solve(R @ (A @ e))
            for _ in range(nu2):
                e = T(e)
            return e
        return spla.LinearOperator(A.shape, matvec=mv, dtype=float)
