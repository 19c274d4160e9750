"""Cut cells of a box-minus-holes domain and cell merging (Section 3).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 3.1 defines the cut cell C_i = C_i ∩ Omega of every grid cell, its
type (empty / regular / irregular), its faces, cut faces and cut boundary B_i,
and the connected components of a cut cell.  Section 3.2 (Algorithm 1) merges
extra components and small cells into neighbours.

The outer boundary must be the grid box itself (grid-aligned, handled by ghost
cells, Section 4.1); holes are closed curves of line segments, circular arcs and
cubic Bezier pieces (the spline boundaries of Section 2) strictly inside the
box, oriented with Omega on their left.

Each cut cell is built from its boundary: the pieces of hole curves inside the
cell ("runs", each entering and leaving through the cell edges) and the pieces
of the cell perimeter inside Omega.  Walking counter-clockwise around the
perimeter from the exit of one run always reaches the entry of the next run,
so runs and perimeter pieces close into loops; each loop bounds one connected
component.  Areas and monomial moments follow from Green's theorem,
    ∬ X^a Y^b dX dY = ∮ X^(a+1)/(a+1) Y^b dY,
in the scaled coordinates X = (x - x_c)/h, Y = (y - y_c)/h about the cell
centre (x_c, y_c).  Line pieces are integrated exactly by Gauss-Legendre,
cubic pieces exactly by 16-point Gauss-Legendre (the integrand is a
polynomial of degree <= 17 in t), arcs by 16-point Gauss-Legendre in the
angle.
"""
from __future__ import annotations

import math
from collections import defaultdict

import numpy as np

MAXDEG = 4                      # moments up to total degree 4 (basis of Pi_4)
MONOS = [(a, d - a) for d in range(MAXDEG + 1) for a in range(d, -1, -1)]
MONO_INDEX = {m: k for k, m in enumerate(MONOS)}

_GL = {n: np.polynomial.legendre.leggauss(n) for n in (4, 8, 16)}


class GeometryError(Exception):
    """The grid does not resolve the geometry (degenerate crossing, a hole
    inside one cell, a component with no neighbour to merge into, ...)."""


# ----------------------------------------------------------------------------
# segments
# ----------------------------------------------------------------------------
def _bezier(seg):
    """Control points of a cubic Bezier segment, p = (x0, y0, ..., x3, y3)."""
    return np.asarray(seg.p[:8], float).reshape(4, 2)


def seg_point(seg, t):
    t = np.asarray(t, float)
    if seg.kind == "line":
        x0, y0, x1, y1 = seg.p
        return x0 + t * (x1 - x0), y0 + t * (y1 - y0)
    if seg.kind == "cubic":
        P = _bezier(seg)
        u = 1.0 - t
        b = [u * u * u, 3 * u * u * t, 3 * u * t * t, t * t * t]
        return (sum(b[k] * P[k, 0] for k in range(4)), sum(b[k] * P[k, 1] for k in range(4)))
    cx, cy, r, t0, t1 = seg.p
    th = t0 + t * (t1 - t0)
    return cx + r * np.cos(th), cy + r * np.sin(th)


def seg_deriv(seg, t):
    t = np.asarray(t, float)
    if seg.kind == "line":
        x0, y0, x1, y1 = seg.p
        return np.full(t.shape, x1 - x0), np.full(t.shape, y1 - y0)
    if seg.kind == "cubic":
        P = _bezier(seg)
        u = 1.0 - t
        d = [3 * u * u, 6 * u * t, 3 * t * t]
        return (sum(d[k] * (P[k + 1, 0] - P[k, 0]) for k in range(3)),
                sum(d[k] * (P[k + 1, 1] - P[k, 1]) for k in range(3)))
    cx, cy, r, t0, t1 = seg.p
    th = t0 + t * (t1 - t0)
    d = t1 - t0
    return -r * d * np.sin(th), r * d * np.cos(th)


def seg_normal(seg, t):
    """Outward unit normal of Omega (Omega lies on the left of the curve)."""
    dx, dy = seg_deriv(seg, t)
    s = np.hypot(dx, dy)
    return dy / s, -dx / s


def _line_params(seg, coord, value):
    """Parameters t in (0,1) where coordinate `coord` (0=x, 1=y) equals value."""
    if seg.kind == "line":
        x0, y0, x1, y1 = seg.p
        a, b = (x0, x1) if coord == 0 else (y0, y1)
        if a == b:
            if a == value:
                raise GeometryError("segment lies on a grid line")
            return []
        t = (value - a) / (b - a)
        return [t] if -1e-15 < t < 1 + 1e-15 else []
    if seg.kind == "cubic":
        # B(t) - value as a polynomial in t (power basis), its real roots,
        # each polished by Newton steps
        c = _bezier(seg)[:, coord]
        poly = np.array([-c[0] + 3 * c[1] - 3 * c[2] + c[3], 3 * c[0] - 6 * c[1] + 3 * c[2],
                         -3 * c[0] + 3 * c[1], c[0] - value])
        scale = np.abs(c).max() + abs(value)
        while len(poly) > 1 and abs(poly[0]) <= 1e-14 * scale:
            poly = poly[1:]
        if len(poly) == 1:
            if abs(poly[0]) <= 1e-14 * scale:
                raise GeometryError("segment lies on a grid line")
            return []
        dpoly = np.polyder(poly)
        out = []
        for z in np.roots(poly):
            if abs(z.imag) > 1e-7:
                continue
            t = float(z.real)
            for _ in range(4):
                d = float(np.polyval(dpoly, t))
                if d == 0.0:
                    break
                t -= float(np.polyval(poly, t)) / d
            if -1e-15 < t < 1 + 1e-15:
                if abs(float(np.polyval(dpoly, t))) < 1e-9 * scale:
                    raise GeometryError("cubic segment tangent to a grid line")
                if not any(abs(t - q) < 1e-13 for q in out):
                    out.append(t)
        return sorted(out)
    cx, cy, r, t0, t1 = seg.p
    cc = cx if coord == 0 else cy
    q = (value - cc) / r
    if abs(q) > 1.0:
        return []
    if abs(abs(q) - 1.0) < 1e-12:
        raise GeometryError("arc tangent to a grid line")
    base = math.acos(q) if coord == 0 else math.asin(q)
    cands = (base, -base) if coord == 0 else (base, math.pi - base)
    lo, hi = min(t0, t1), max(t0, t1)
    out = []
    for th in cands:
        k0 = math.floor((lo - th) / (2 * math.pi)) - 1
        for k in range(k0, k0 + 4):
            tt = th + 2 * math.pi * k
            if lo - 1e-15 < tt < hi + 1e-15:
                out.append((tt - t0) / (t1 - t0))
    return out


# ----------------------------------------------------------------------------
# moments by Green's theorem
# ----------------------------------------------------------------------------
def _curve_moments(seg, ta, tb, xc, yc, h):
    """∮ X^(a+1)/(a+1) Y^b dY along seg for t in [ta, tb], all (a,b) in MONOS,
    scaled coordinates about (xc, yc)."""
    n = 4 if seg.kind == "line" else 16
    s, w = _GL[n]
    t = 0.5 * (tb - ta) * s + 0.5 * (ta + tb)
    wt = 0.5 * (tb - ta) * w
    x, y = seg_point(seg, t)
    _, dy = seg_deriv(seg, t)
    X = (x - xc) / h
    Y = (y - yc) / h
    dY = dy / h
    out = np.empty(len(MONOS))
    for k, (a, b) in enumerate(MONOS):
        out[k] = np.sum(wt * X ** (a + 1) / (a + 1) * Y ** b * dY)
    return out


def _edge_moments(side, s0, s1):
    """Contribution of a perimeter piece; side 1 = right (X=1/2, Y = s - 1/2),
    side 3 = left (X=-1/2, Y = 1/2 - s), s = position along the side in [0,1]
    in counter-clockwise direction.  Horizontal sides have dY = 0."""
    out = np.zeros(len(MONOS))
    if side == 1:
        Xv, Ya, Yb = 0.5, s0 - 0.5, s1 - 0.5
    elif side == 3:
        Xv, Ya, Yb = -0.5, 0.5 - s0, 0.5 - s1
    else:
        return out
    for k, (a, b) in enumerate(MONOS):
        out[k] = Xv ** (a + 1) / (a + 1) * (Yb ** (b + 1) - Ya ** (b + 1)) / (b + 1)
    return out


def full_cell_moments():
    """Moments of the unit square [-1/2,1/2]^2."""
    out = np.zeros(len(MONOS))
    for k, (a, b) in enumerate(MONOS):
        ia = 0.0 if a % 2 else 1.0 / ((a + 1) * 2 ** a)
        ib = 0.0 if b % 2 else 1.0 / ((b + 1) * 2 ** b)
        out[k] = ia * ib
    return out


def shift_moments(mom, dx, dy):
    """Moments about a centre shifted by (-dx, -dy) cells: returns
    ∬ (X+dx)^a (Y+dy)^b given ∬ X^p Y^q (binomial expansion)."""
    if dx == 0 and dy == 0:
        return mom.copy()
    out = np.zeros(len(MONOS))
    for k, (a, b) in enumerate(MONOS):
        s = 0.0
        for p in range(a + 1):
            for q in range(b + 1):
                s += (math.comb(a, p) * math.comb(b, q) * dx ** (a - p) * dy ** (b - q)
                      * mom[MONO_INDEX[(p, q)]])
        out[k] = s
    return out


# ----------------------------------------------------------------------------
# cut cells on one grid
# ----------------------------------------------------------------------------
class Component:
    __slots__ = ("cell", "mom", "faces", "bpieces", "loops", "key", "root", "absorbed", "vtot")

    def __init__(self, cell, mom, faces, bpieces, loops, key):
        self.cell = cell          # grid cell (i, j)
        self.mom = mom            # moments about the centre of `cell`, scaled (vol = mom[0])
        self.faces = faces        # list of (facekey, lo, hi)
        self.bpieces = bpieces    # list of (curve, seg, ta, tb)
        self.loops = loops        # list of loops; loop = list of ('run', pieces) / ('edge', side, s0, s1)
        self.key = key            # ordering key within its cell
        self.root = self          # union-find parent
        self.absorbed = []        # components merged into this one
        self.vtot = float(mom[0]) # total volume of the region rooted here


def _find(c):
    while c.root is not c:
        c.root = c.root.root
        c = c.root
    return c


def _face_key(i, j, side):
    """Face keys: ('v', k, j) = x = x0 + k h between cells (k-1, j) and (k, j);
    ('h', i, l) = y = y0 + l h between cells (i, l-1) and (i, l)."""
    if side == 0:
        return ("h", i, j)
    if side == 1:
        return ("v", i + 1, j)
    if side == 2:
        return ("h", i, j + 1)
    return ("v", i, j)


def _face_interval(side, s0, s1):
    """Map a perimeter interval on `side` (CCW position in [0,1]) to the
    face's own increasing coordinate (x for horizontal, y for vertical)."""
    if side in (0, 1):
        return (s0, s1)
    return (1.0 - s1, 1.0 - s0)


class CutGrid:
    """All cut cells of one level after Algorithm 1.

    Attributes (arrays indexed [j, i]):
      active   -- cell is in C^h_eps
      regular  -- C_i equals the full grid cell
      volfrac  -- ||C_i|| / h^2
    ``cells[(i, j)]`` for active irregular cells: dict(mom, bpieces, members)
    ``owner[(i, j)]`` for grid cells whose content was merged elsewhere.
    """

    def __init__(self, grid, curves, eps):
        self.grid = grid
        self.curves = curves
        self.eps = float(eps)
        self.nx, self.ny, self.h = grid.nx, grid.ny, grid.h
        self._check_box()
        self._cut()
        self._merge()

    # -- outer box ------------------------------------------------------------
    def _check_box(self):
        g = self.grid
        x1, y1 = g.x0 + g.nx * g.h, g.y0 + g.ny * g.h
        want = [(g.x0, g.y0, x1, g.y0), (x1, g.y0, x1, y1), (x1, y1, g.x0, y1), (g.x0, y1, g.x0, g.y0)]
        box = self.curves[0]
        if len(box) != 4 or any(s.kind != "line" for s in box):
            raise GeometryError("the outer curve must be the grid box (4 line segments)")
        for s, w in zip(box, want):
            if any(abs(p - q) > 1e-12 * max(1.0, abs(q)) for p, q in zip(s.p, w)):
                raise GeometryError("the outer curve must be the counter-clockwise grid box")
        # side order bottom, right, top, left
        self.box_bc = [(s.bc, s.alpha1, s.alpha2) for s in box]
        # periodic sides come in opposite pairs (Sec. 4.1), and only on the box
        for a, b in ((0, 2), (1, 3)):
            if (box[a].bc == "P") != (box[b].bc == "P"):
                raise GeometryError("periodic box sides must come in opposite pairs")
        if any(s.bc == "P" for c in self.curves[1:] for s in c):
            raise GeometryError("periodic conditions apply to box sides only")

    # -- crossings, runs, loops -------------------------------------------------
    def _cut(self):
        g = self.grid
        h, nx, ny = g.h, g.nx, g.ny
        runs = defaultdict(list)            # cell -> list of runs
        self.hole_nocross = []
        for ci, curve in enumerate(self.curves[1:], start=1):
            pieces = []                      # (seg, ta, tb, start_crossing or None)
            ncross = 0
            for si, seg in enumerate(curve):
                xs, ys = seg_point(seg, np.linspace(0, 1, 65))
                if seg.kind == "cubic":            # the control polygon bounds the curve
                    xs, ys = np.append(xs, _bezier(seg)[:, 0]), np.append(ys, _bezier(seg)[:, 1])
                kx = range(max(0, int(math.floor((xs.min() - g.x0) / h)) - 1),
                           min(nx, int(math.ceil((xs.max() - g.x0) / h)) + 1) + 1)
                ky = range(max(0, int(math.floor((ys.min() - g.y0) / h)) - 1),
                           min(ny, int(math.ceil((ys.max() - g.y0) / h)) + 1) + 1)
                cr = []
                for k in kx:
                    for t in _line_params(seg, 0, g.x0 + k * h):
                        cr.append((t, "v", k))
                for l in ky:
                    for t in _line_params(seg, 1, g.y0 + l * h):
                        cr.append((t, "h", l))
                cr.sort()
                for t, _, _ in cr:
                    if t < 1e-12 or t > 1 - 1e-12:
                        raise GeometryError("curve vertex on a grid line")
                for a in range(len(cr) - 1):
                    if cr[a + 1][0] - cr[a][0] < 1e-12:
                        raise GeometryError("curve passes through a grid vertex")
                ncross += len(cr)
                bps = [(0.0, None)] + [(t, (kind, k)) for t, kind, k in cr] + [(1.0, None)]
                for a in range(len(bps) - 1):
                    pieces.append((si, bps[a][0], bps[a + 1][0], bps[a][1], bps[a + 1][1]))
            if ncross == 0:
                raise GeometryError("a hole lies inside a single cell")
            # cell of each piece
            def cell_of(p):
                seg = curve[p[0]]
                xm, ym = seg_point(seg, 0.5 * (p[1] + p[2]))
                return (int(math.floor((float(xm) - g.x0) / h)), int(math.floor((float(ym) - g.y0) / h)))
            # rotate so that the list starts at a crossing
            start = next(k for k, p in enumerate(pieces) if p[3] is not None)
            pieces = pieces[start:] + pieces[:start]
            cur = None
            for p in pieces:
                if p[3] is not None:          # a crossing starts a new run
                    cell = cell_of(p)
                    if not (0 <= cell[0] < nx and 0 <= cell[1] < ny):
                        raise GeometryError("hole leaves the box")
                    cur = {"cell": cell, "pieces": [], "entry": None, "exit": None, "curve": ci}
                    cur["entry"] = self._tau(cell, curve[p[0]], p[1], p[3])
                    runs[cell].append(cur)
                cur["pieces"].append((ci, p[0], p[1], p[2]))
                if p[4] is not None:
                    cur["exit"] = self._tau(cur["cell"], curve[p[0]], p[2], p[4])
        self.runs = runs

    def _tau(self, cell, seg, t, line):
        """Perimeter coordinate in [0,4) of a crossing on the edge of `cell`."""
        g = self.grid
        i, j = cell
        x, y = (float(v) for v in seg_point(seg, t))
        X0, Y0 = g.x0 + i * g.h, g.y0 + j * g.h
        kind, k = line
        if kind == "h":
            if k == j:
                return (x - X0) / g.h
            if k == j + 1:
                return 2.0 + (X0 + g.h - x) / g.h
        else:
            if k == i + 1:
                return 1.0 + (y - Y0) / g.h
            if k == i:
                return 3.0 + (Y0 + g.h - y) / g.h
        raise GeometryError("crossing not on the cell perimeter")

    def _loops(self, cell, runs):
        order = sorted(range(len(runs)), key=lambda r: runs[r]["entry"])
        nxt = {}
        for r in order:
            tout = runs[r]["exit"]
            best = min(order, key=lambda q: (runs[q]["entry"] - tout) % 4.0)
            nxt[r] = best
        seen = set()
        loops = []
        for r0 in order:
            if r0 in seen:
                continue
            loop = []
            r = r0
            while r not in seen:
                seen.add(r)
                loop.append(("run", runs[r]["pieces"]))
                tout = runs[r]["exit"]
                q = nxt[r]
                tin = runs[q]["entry"]
                span = (tin - tout) % 4.0
                # perimeter pieces from tout to tin, split at corners
                pos = tout
                remaining = span
                while remaining > 1e-15:
                    side = int(math.floor(pos + 1e-15)) % 4
                    s0 = pos - math.floor(pos + 1e-15)
                    if s0 < 0:
                        s0 = 0.0
                    step = min(remaining, 1.0 - s0)
                    loop.append(("edge", side, s0, s0 + step))
                    remaining -= step
                    pos = (pos + step) % 4.0
                r = q
            loops.append((runs[r0]["entry"], loop))
        return loops

    def _component_from_loop(self, cell, loop):
        i, j = cell
        g = self.grid
        xc, yc = g.x0 + (i + 0.5) * g.h, g.y0 + (j + 0.5) * g.h
        mom = np.zeros(len(MONOS))
        faces, bpieces = [], []
        for item in loop:
            if item[0] == "run":
                for (ci, si, ta, tb) in item[1]:
                    mom += _curve_moments(self.curves[ci][si], ta, tb, xc, yc, g.h)
                    bpieces.append((ci, si, ta, tb))
            else:
                _, side, s0, s1 = item
                mom += _edge_moments(side, s0, s1)
                lo, hi = _face_interval(side, s0, s1)
                faces.append((_face_key(i, j, side), lo, hi))
        return mom, faces, bpieces

    # -- Algorithm 1 -----------------------------------------------------------
    def _merge(self):
        g = self.grid
        nx, ny = g.nx, g.ny
        inside = self._inside_mask()
        comps = {}                           # cell -> list of Component (cut cells only)
        for cell, rlist in self.runs.items():
            lst = []
            for key, loop in self._loops(cell, rlist):
                mom, faces, bp = self._component_from_loop(cell, loop)
                if mom[0] <= 0.0:
                    raise GeometryError("negatively oriented loop (hole inside a cell)")
                lst.append(Component(cell, mom, faces, bp, [loop], key))
            lst.sort(key=lambda c: c.key)
            comps[cell] = lst
        self.cutcells = set(comps)
        for cell in comps:
            inside[cell[1], cell[0]] = False
        full = {}                            # regular cells that become merge targets

        def full_comp(cell):
            if cell not in full:
                i, j = cell
                faces = [(_face_key(i, j, s), 0.0, 1.0) for s in range(4)]
                full[cell] = Component(cell, full_cell_moments(), faces, [], [], 0.0)
            return full[cell]

        def comps_of(cell):
            if cell in comps:
                return comps[cell]
            i, j = cell
            if 0 <= i < nx and 0 <= j < ny and inside[j, i]:
                return [full_comp(cell)]
            return []

        def neighbours(cell):
            i, j = cell
            return [(i - 1, j), (i + 1, j), (i, j - 1), (i, j + 1)]

        def touching(c, other_cell):
            """Components of other_cell sharing a positive-length face piece with c."""
            out = []
            for oc in comps_of(other_cell):
                hit = False
                for fk, lo, hi in c.faces:
                    for fk2, lo2, hi2 in oc.faces:
                        if fk == fk2 and min(hi, hi2) - max(lo, lo2) > 1e-9:
                            hit = True
                            break
                    if hit:
                        break
                if hit:
                    out.append(oc)
            return out

        def absorb(target, src):
            target.absorbed.append(src)
            src.root = target

        # total volume (in units of h^2) is tracked on union-find roots
        for lst in comps.values():
            for c in lst:
                c.vtot = float(c.mom[0])
        # lines 2-7: cells with several components
        for j in range(ny):
            for i in range(nx):
                cell = (i, j)
                lst = comps.get(cell)
                if not lst or len(lst) < 2:
                    continue
                m = max(range(len(lst)), key=lambda k: (lst[k].mom[0], -k))
                for k, ck in enumerate(lst):
                    if k == m:
                        continue
                    rk = _find(ck)
                    best, bestval = None, None
                    for nb in neighbours(cell):
                        for oc in touching(ck, nb):
                            ro = _find(oc)
                            if ro is rk:
                                continue
                            val = abs(ro.vtot + rk.vtot - 1.0)
                            if bestval is None or val < bestval - 1e-12:
                                best, bestval = ro, val
                    if best is None:
                        raise GeometryError("a minor component has no neighbour to merge into")
                    absorb(best, rk)
                    best.vtot += rk.vtot
        # lines 8-11: small cells
        self.removed = set()
        main = {}
        for cell, lst in comps.items():
            m = max(range(len(lst)), key=lambda k: (lst[k].mom[0], -k))
            main[cell] = lst[m]

        def cell_root(cell):
            if cell in main:
                return _find(main[cell])
            return _find(full_comp(cell))

        def region_members(root):
            out, stack = [], [root]
            while stack:
                c = stack.pop()
                out.append(c)
                stack.extend(c.absorbed)
            return out

        for j in range(ny):
            for i in range(nx):
                cell = (i, j)
                if cell not in main or cell in self.removed:
                    continue
                r = cell_root(cell)
                if r.cell != cell:
                    raise GeometryError("main component absorbed elsewhere")
                if r.vtot >= self.eps:
                    continue
                members = region_members(r)
                best, bestval = None, None
                for nb in neighbours(cell):
                    if not (0 <= nb[0] < nx and 0 <= nb[1] < ny) or nb in self.removed:
                        continue
                    if nb not in main and not inside[nb[1], nb[0]]:
                        continue
                    rn = cell_root(nb)
                    if rn.cell != nb:
                        continue
                    hit = False
                    for c in members:
                        for gc in neighbours(c.cell):
                            for oc in touching(c, gc):
                                if _find(oc) is rn:
                                    hit = True
                                    break
                            if hit:
                                break
                        if hit:
                            break
                    if not hit:
                        continue
                    val = abs(rn.vtot + r.vtot - 1.0)
                    if bestval is None or val < bestval - 1e-12:
                        best, bestval = rn, val
                if best is None:
                    raise GeometryError("a small cell has no neighbour to merge into")
                absorb(best, r)
                best.vtot += r.vtot
                self.removed.add(cell)
        # results
        self.active = inside.copy()
        for cell in comps:
            if cell not in self.removed:
                self.active[cell[1], cell[0]] = True
        self.regular = inside.copy()
        self.cells = {}
        roots = {}
        for cell in list(main) + list(full):
            if cell in self.removed:
                continue
            r = cell_root(cell)
            roots[cell] = r
        for cell, r in roots.items():
            members = region_members(r)
            if len(members) == 1 and cell in full:
                continue                      # untouched regular cell
            self.regular[cell[1], cell[0]] = False
            mom = np.zeros(len(MONOS))
            bp = []
            for c in members:
                mom += shift_moments(c.mom, c.cell[0] - cell[0], c.cell[1] - cell[1])
                bp.extend(c.bpieces)
            self.cells[cell] = {"mom": mom, "bpieces": bp, "members": members}
        # owner map: grid cells whose content lives in another cell
        self.owner = {}
        for cell in self.removed:
            self.owner[cell] = _find(main[cell]).cell
        self.volfrac = np.where(self.regular, 1.0, 0.0)
        for cell, d in self.cells.items():
            self.volfrac[cell[1], cell[0]] = d["mom"][0]

    def _inside_mask(self):
        """Cells whose centre lies in Omega (box minus holes), by counting
        crossings of the horizontal line through the centres."""
        g = self.grid
        nx, ny, h = g.nx, g.ny, g.h
        inside = np.ones((ny, nx), bool)
        xcen = g.x0 + (np.arange(nx) + 0.5) * h
        for curve in self.curves[1:]:
            for j in range(ny):
                yc = g.y0 + (j + 0.5) * h
                xs = []
                for seg in curve:
                    for t in _line_params(seg, 1, yc):
                        if 0.0 <= t < 1.0:
                            xs.append(float(seg_point(seg, t)[0]))
                if not xs:
                    continue
                xs.sort()
                # parity of crossings to the right of each centre
                cnt = len(xs) - np.searchsorted(np.array(xs), xcen, side="right")
                inside[j] &= (cnt % 2 == 0)
        return inside

    # -- convenience ------------------------------------------------------------
    def cell_moments(self, cell):
        """Scaled moments ∬ X^a Y^b / h^2-area units of an active cell about
        the centre of its grid cell (volume = entry 0)."""
        if cell in self.cells:
            return self.cells[cell]["mom"]
        return full_cell_moments()

    def is_active(self, i, j):
        return 0 <= i < self.nx and 0 <= j < self.ny and bool(self.active[j, i])

    def is_regular(self, i, j):
        return 0 <= i < self.nx and 0 <= j < self.ny and bool(self.regular[j, i])

    def boundary_length(self, cell):
        """||B_i|| of an irregular cell (physical length)."""
        L = 0.0
        s, w = _GL[16]
        for ci, si, ta, tb in self.cells[cell]["bpieces"]:
            seg = self.curves[ci][si]
            t = 0.5 * (tb - ta) * s + 0.5 * (ta + tb)
            dx, dy = seg_deriv(seg, t)
            L += float(np.sum(0.5 * (tb - ta) * w * np.hypot(dx, dy)))
        return L
