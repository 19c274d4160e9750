"""Cell averages and boundary averages of given functions (eqs. (4.1)-(4.2)).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Regular cells use an 8x8 tensor Gauss-Legendre rule.  Irregular (cut or
merged) cells use Green's theorem, ∬ f = ∮ F dy with F(x, y) the integral of
f(., y) from the cell-centre abscissa to x, evaluated by Gauss-Legendre along
every boundary piece (16 points on curve pieces, 8 on cell edges) and by an
inner 16-point rule for F.  Boundary averages use 16-point Gauss-Legendre in
the curve parameter, weighted by arc length.
"""
from __future__ import annotations

import numpy as np

from .geometry import _GL, seg_deriv, seg_normal, seg_point

_G8 = _GL[8]
_G16 = _GL[16]


def _antideriv(func, x, y, xr):
    s, w = _G16
    x = np.asarray(x, float)[..., None]
    y = np.asarray(y, float)[..., None]
    half = 0.5 * (x - xr)
    pts = xr + half * (1.0 + s)
    return np.sum(w * func(pts, np.broadcast_to(y, pts.shape)), axis=-1) * half[..., 0]


def _component_integral(level, comp, func):
    """∬ func over one component (physical units)."""
    g = level.grid
    h = g.h
    i, j = comp.cell
    X0, Y0 = g.x0 + i * h, g.y0 + j * h
    xr = X0 + 0.5 * h
    if not comp.loops:                  # a full grid cell (regular cell that absorbed a neighbour)
        s, w = _G8
        xs = X0 + (0.5 + 0.5 * s) * h
        ys = Y0 + (0.5 + 0.5 * s) * h
        return float(0.25 * h * h * np.einsum("a,b,ab->", w, w, func(xs[:, None], ys[None, :])))
    total = 0.0
    for loop in comp.loops:
        for item in loop:
            if item[0] == "run":
                for ci, si, ta, tb in item[1]:
                    seg = level.curves[ci][si]
                    s, w = _G16
                    t = 0.5 * (tb - ta) * s + 0.5 * (ta + tb)
                    x, y = seg_point(seg, t)
                    _, dy = seg_deriv(seg, t)
                    total += float(np.sum(0.5 * (tb - ta) * w * _antideriv(func, x, y, xr) * dy))
            else:
                _, side, s0, s1 = item
                if side not in (1, 3):
                    continue
                s, w = _G8
                if side == 1:
                    x = X0 + h
                    ya, yb = Y0 + s0 * h, Y0 + s1 * h
                else:
                    x = X0
                    ya, yb = Y0 + (1.0 - s0) * h, Y0 + (1.0 - s1) * h
                y = 0.5 * (yb - ya) * s + 0.5 * (ya + yb)
                total += float(np.sum(0.5 * (yb - ya) * w * _antideriv(func, np.full(y.shape, x), y, xr)))
    return total


def cell_averages(level, func):
    """<func>_i for every active cell of `level` (compact order)."""
    g = level.grid
    h = g.h
    s, w = _G8
    out = np.empty(level.n)
    reg = level.cg.regular[level.cells_j, level.cells_i]
    ii, jj = level.cells_i[reg], level.cells_j[reg]
    xs = g.x0 + (ii[:, None] + 0.5 + 0.5 * s[None, :]) * h
    ys = g.y0 + (jj[:, None] + 0.5 + 0.5 * s[None, :]) * h
    vals = func(xs[:, :, None], ys[:, None, :])
    out[reg] = 0.25 * np.einsum("a,b,nab->n", w, w, vals)
    for cell, d in level.cg.cells.items():
        k = level.idx[cell[1], cell[0]]
        integ = sum(_component_integral(level, c, func) for c in d["members"])
        out[k] = integ / (d["mom"][0] * h * h)
    return out


def _bc_value(seg, sol, x, y, nx, ny):
    u = sol.u(x, y)
    if seg.bc == "P":                  # periodic box sides carry no data
        return np.zeros_like(u)
    dn = sol.ux(x, y) * nx + sol.uy(x, y) * ny
    if seg.bc == "D":
        return u
    if seg.bc == "N":
        return dn
    return seg.alpha1 * u + seg.alpha2 * dn


def boundary_data(level, sol):
    """The vector g of eq. (4.19): box-face averages of N u, then
    <<N u>>_{B_i} of every irregular cell, in the level's layout."""
    g = np.zeros(level.n_g)
    gr = level.grid
    h, nx, ny = gr.h, gr.nx, gr.ny
    s, w = _G8
    box = level.curves[0]
    for side in range(4):
        seg = box[side]
        cnt = nx if side in (0, 2) else ny
        for k in range(cnt):
            if side == 0:
                x = gr.x0 + (k + 0.5 + 0.5 * s) * h; y = np.full(8, gr.y0); n = (0.0, -1.0)
            elif side == 2:
                x = gr.x0 + (k + 0.5 + 0.5 * s) * h; y = np.full(8, gr.y0 + ny * h); n = (0.0, 1.0)
            elif side == 3:
                y = gr.y0 + (k + 0.5 + 0.5 * s) * h; x = np.full(8, gr.x0); n = (-1.0, 0.0)
            else:
                y = gr.y0 + (k + 0.5 + 0.5 * s) * h; x = np.full(8, gr.x0 + nx * h); n = (1.0, 0.0)
            g[level.face_index(side, k)] = 0.5 * np.sum(w * _bc_value(seg, sol, x, y, n[0], n[1]))
    s16, w16 = _G16
    for cell in level.irregular:
        tot = 0.0
        length = 0.0
        for ci, si, ta, tb in level.cg.cells[cell]["bpieces"]:
            seg = level.curves[ci][si]
            t = 0.5 * (tb - ta) * s16 + 0.5 * (ta + tb)
            x, y = seg_point(seg, t)
            dx, dy = seg_deriv(seg, t)
            ds = 0.5 * (tb - ta) * w16 * np.hypot(dx, dy)
            n0, n1 = seg_normal(seg, t)
            tot += float(np.sum(ds * _bc_value(seg, sol, x, y, n0, n1)))
            length += float(np.sum(ds))
        g[level.g_irr[cell]] = tot / length
    return g


def rhs(level, sol):
    """b = f - N g (eq. (4.19)) and the pieces (f, g)."""
    f = cell_averages(level, sol.f)
    gv = boundary_data(level, sol)
    return f - level.N @ gv, f, gv
