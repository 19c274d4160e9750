"""Pins of the oracle's cut cells and Algorithm 1 against closed forms and an
independent polygon clipper (Section 3)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.geometry import CutGrid, GeometryError, MONOS


def _clip_convex(poly, x0, y0, x1, y1):
    """Sutherland-Hodgman clip of polygon `poly` (list of points) to a box."""
    def clip(pts, inside, inter):
        out = []
        for k in range(len(pts)):
            p, q = pts[k - 1], pts[k]
            if inside(q):
                if not inside(p):
                    out.append(inter(p, q))
                out.append(q)
            elif inside(p):
                out.append(inter(p, q))
        return out

    def ix(X):
        return lambda p, q: (X, p[1] + (q[1] - p[1]) * (X - p[0]) / (q[0] - p[0]))

    def iy(Y):
        return lambda p, q: (p[0] + (q[0] - p[0]) * (Y - p[1]) / (q[1] - p[1]), Y)
    pts = poly
    for ins, it in ((lambda p: p[0] >= x0, ix(x0)), (lambda p: p[0] <= x1, ix(x1)),
                    (lambda p: p[1] >= y0, iy(y0)), (lambda p: p[1] <= y1, iy(y1))):
        if pts:
            pts = clip(pts, ins, it)
    return pts


def _area(pts):
    return 0.5 * sum(pts[k - 1][0] * pts[k][1] - pts[k][0] * pts[k - 1][1] for k in range(len(pts)))


def _polygon_problem(n, verts_ccw):
    segs = []
    cw = list(reversed(verts_ccw))
    for k in range(len(cw)):
        p, q = cw[k], cw[(k + 1) % len(cw)]
        segs.append(W.Segment("line", (p[0], p[1], q[0], q[1])))
    return W.Grid(0.0, 0.0, 1.0 / n, n, n), [W.box_curve(0, 0, 1, 1), segs]


@pytest.mark.parametrize("n", [16, 32, 64])
def test_cut_cell_areas_match_polygon_clipping(n):
    """Before merging, each cut cell's area equals h^2 minus the area of the
    (convex) hole clipped to the cell."""
    ang = [0.37 + k * 2 * math.pi / 5 for k in range(5)]
    verts = [(0.5 + 0.27 * math.cos(t), 0.48 + 0.27 * math.sin(t)) for t in ang]
    grid, curves = _polygon_problem(n, verts)
    cg = CutGrid(grid, curves, eps=1e-9)
    h = grid.h
    own = {}                                       # components grouped by their grid cell
    for d in cg.cells.values():
        for c in d["members"]:
            own[c.cell] = own.get(c.cell, 0.0) + c.mom[0]
    assert set(own) >= set(cg.cutcells)
    for (i, j) in cg.cutcells:
        clip = _clip_convex(verts, i * h, j * h, (i + 1) * h, (j + 1) * h)
        hole = _area(clip) if len(clip) >= 3 else 0.0
        assert own[(i, j)] * h * h == pytest.approx(h * h - hole, abs=1e-15)


@pytest.mark.parametrize("maker,n", [(W.unit_disk_config, 64), (W.three_disks_config, 128),
                                     (W.star_config, 128)])
def test_volumes_and_first_moments_sum_to_domain(maker, n):
    P = maker(0, n)
    cg = CutGrid(P.grid, P.curves, P.eps)
    h = P.grid.h
    # eq. (3.5): the merged cells partition Omega
    area = cg.volfrac.sum() * h * h
    if "disks" in P.meta:
        exact = 1.0 - sum(math.pi * r * r for _, _, r in P.meta["disks"])
        mx = 0.5 - sum(math.pi * r * r * cx for cx, _, r in P.meta["disks"])
    elif maker is W.unit_disk_config:
        exact = 1.0 - math.pi * 0.04
        mx = 0.5 - math.pi * 0.04 * 0.5
    else:
        exact = mx = None
    if exact is not None:
        assert area == pytest.approx(exact, abs=1e-13)
        # first moment int x dA: regular cells at their centres, cut cells via moments
        tot = 0.0
        jj, ii = np.nonzero(cg.regular)
        tot += np.sum((ii + 0.5) * h) * h * h
        kx = MONOS.index((1, 0))
        for (i, j), d in cg.cells.items():
            tot += ((i + 0.5) * h * d["mom"][0] + h * d["mom"][kx]) * h * h
        assert tot == pytest.approx(mx, abs=1e-13)
    # Algorithm 1 postconditions
    act = cg.active
    assert np.all(cg.volfrac[act] >= P.eps - 1e-15)
    assert not np.any(cg.volfrac[~act] > 0)


def test_star_area_closed_form():
    """The star hole is a polygon with arcs; its area follows from Green's
    theorem on the curve itself, independently of the cut cells."""
    P = W.star_config(0, 128)
    hole = 0.0
    for s in P.curves[1]:
        if s.kind == "line":
            x0, y0, x1, y1 = s.p
            hole += 0.5 * (x0 * y1 - x1 * y0)
        else:
            cx, cy, r, t0, t1 = s.p
            hole += 0.5 * (r * r * (t1 - t0) + cx * r * (math.sin(t1) - math.sin(t0))
                           - cy * r * (math.cos(t1) - math.cos(t0)))
    hole = -hole                               # the hole is traversed clockwise
    cg = CutGrid(P.grid, P.curves, P.eps)
    assert cg.volfrac.sum() * P.grid.h ** 2 == pytest.approx(1.0 - hole, abs=1e-13)


def test_merging_removes_small_cells():
    P = W.unit_disk_config(0, 64)
    cg = CutGrid(P.grid, P.curves, P.eps)
    assert cg.removed, "the disk at 64^2 has cells below eps h^2"
    for cell in cg.removed:
        own = cg.owner[cell]
        assert abs(own[0] - cell[0]) + abs(own[1] - cell[1]) == 1
        assert cg.active[own[1], own[0]] and not cg.active[cell[1], cell[0]]


def test_hole_inside_one_cell_is_rejected():
    grid = W.Grid(0.0, 0.0, 1.0 / 8, 8, 8)
    curves = [W.box_curve(0, 0, 1, 1), W.disk_hole(0.5 + 1 / 16, 0.5 + 1 / 16, 0.02)]
    with pytest.raises(GeometryError):
        CutGrid(grid, curves, 0.08)


def _bezier_area_and_moment(curve):
    """Signed area and first x-moment enclosed by a closed curve of cubic
    Bezier pieces, by exact polynomial integration of Green's theorem
    (x dy and x^2/2 dy) in the power basis of each piece's control points."""
    from numpy.polynomial import polynomial as Pn
    to_power = np.array([[1, 0, 0, 0], [-3, 3, 0, 0], [3, -6, 3, 0], [-1, 3, -3, 1]], float)
    area = mom = 0.0
    for sg in curve:
        c = np.array(sg.p, float).reshape(4, 2)
        x, y = to_power @ c[:, 0], to_power @ c[:, 1]
        dy = Pn.polyder(y)
        for integrand, acc in ((Pn.polymul(x, dy), "a"), (0.5 * Pn.polymul(Pn.polymul(x, x), dy), "m")):
            F = Pn.polyint(integrand)
            v = Pn.polyval(1.0, F) - Pn.polyval(0.0, F)
            if acc == "a":
                area += v
            else:
                mom += v
    return area, mom


@pytest.mark.parametrize("seed,n", [(0, 64), (1, 128), (2, 96)])
def test_bezier_hole_volumes_and_first_moment(seed, n):
    """Cubic Bezier boundary pieces (Section 2's splines): the cut cells
    partition the unit square minus the hole, whose area and first moment
    follow exactly from its control points."""
    P = W.bezier_config(seed, n)
    cg = CutGrid(P.grid, P.curves, P.eps)
    h = P.grid.h
    a_hole, m_hole = _bezier_area_and_moment(P.curves[1])     # clockwise: negative
    assert cg.volfrac.sum() * h * h == pytest.approx(1.0 + a_hole, abs=1e-13)
    tot = 0.0
    jj, ii = np.nonzero(cg.regular)
    tot += np.sum((ii + 0.5) * h) * h * h
    kx = MONOS.index((1, 0))
    for (i, j), d in cg.cells.items():
        tot += ((i + 0.5) * h * d["mom"][0] + h * d["mom"][kx]) * h * h
    assert tot == pytest.approx(0.5 + m_hole, abs=1e-13)
    act = cg.active
    assert np.all(cg.volfrac[act] >= P.eps - 1e-15)


def test_bezier_crossings_are_roots():
    """Every grid-line crossing of a cubic piece is a root of its coordinate
    polynomial to rounding, and no crossing is missed (sign changes of the
    coordinate minus the grid value on a fine sampling)."""
    from oracle.geometry import _line_params, seg_point
    P = W.bezier_config(3, 64)
    h = P.grid.h
    for sg in P.curves[1]:
        t = np.linspace(0.0, 1.0, 4001)
        x, y = seg_point(sg, t)
        for coord, vals in ((0, x), (1, y)):
            for k in range(65):
                v = k * h
                got = _line_params(sg, coord, v)
                for tt in got:
                    xv, yv = seg_point(sg, tt)
                    assert abs((xv if coord == 0 else yv) - v) <= 1e-14
                changes = int(np.sum(np.sign(vals[1:] - v) != np.sign(vals[:-1] - v)))
                assert len(got) == changes
