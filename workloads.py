"""Seeded synthetic inputs shared by the oracle-side tests and the GPU-side runs.

This module only describes problems: grids, boundary curves with their boundary
conditions, elliptic coefficients and manufactured solutions.  It holds none of
the discretisation, geometry or solver arithmetic; each side (the oracle under
``oracle/`` and the HIP library) derives everything else itself.

Problem statement (Section 1, eqs. (1.1)-(1.2)): find u with
    a u_xx + b u_xy + c u_yy = f  in Omega,   N u = g  on dOmega,
with b^2 - 4ac < 0 and N the identity (Dirichlet), d/dn (Neumann) or
alpha1 + alpha2 d/dn (Robin).  Omega is a square box minus holes; every
boundary curve is closed and oriented with Omega on its left (Section 2),
so the box is traversed counter-clockwise and each hole clockwise.

Segment kinds
  ('line',  (x0, y0, x1, y1))
  ('arc',   (cx, cy, r, theta0, theta1))   signed sweep theta1 - theta0
  ('cubic', (x0, y0, x1, y1, x2, y2, x3, y3))   Bezier control points
Each segment carries its boundary condition: bc in {'D', 'N', 'R'} and the
Robin coefficients (alpha1, alpha2); box sides may also be periodic ('P', in
opposite pairs).  The outward normal of Omega at a point
with tangent (x', y') is (y', -x') / |(x', y')|.

Random draws use numpy.random.default_rng(seed) (PCG64); the draw order is the
order of the statements below and must not change, since stored expected
values depend on it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BC_DIRICHLET, BC_NEUMANN, BC_ROBIN, BC_PERIODIC = "D", "N", "R", "P"


@dataclass(frozen=True)
class Segment:
    kind: str                      # 'line' or 'arc'
    p: tuple                       # see module docstring
    bc: str = BC_DIRICHLET
    alpha1: float = 1.0
    alpha2: float = 0.0


@dataclass
class Grid:
    x0: float
    y0: float
    h: float
    nx: int
    ny: int


@dataclass
class Problem:
    name: str
    grid: Grid
    curves: list                   # list of list[Segment]; curves[0] is the outer box
    a: float
    b: float
    c: float
    solution: object               # provides u, ux, uy, f (vectorised over numpy arrays)
    eps: float = 0.08
    meta: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------
# manufactured solutions
# ----------------------------------------------------------------------------
class SineModes:
    """u = sum_m A_m sin(k1_m pi x) sin(k2_m pi y)."""

    def __init__(self, modes, a, b, c):
        self.modes = [(int(k1), int(k2), float(A)) for k1, k2, A in modes]
        self.a, self.b, self.c = float(a), float(b), float(c)

    def u(self, x, y):
        x = np.asarray(x, float); y = np.asarray(y, float)
        s = np.zeros(np.broadcast(x, y).shape)
        for k1, k2, A in self.modes:
            s = s + A * np.sin(k1 * math.pi * x) * np.sin(k2 * math.pi * y)
        return s

    def ux(self, x, y):
        x = np.asarray(x, float); y = np.asarray(y, float)
        s = np.zeros(np.broadcast(x, y).shape)
        for k1, k2, A in self.modes:
            s = s + A * k1 * math.pi * np.cos(k1 * math.pi * x) * np.sin(k2 * math.pi * y)
        return s

    def uy(self, x, y):
        x = np.asarray(x, float); y = np.asarray(y, float)
        s = np.zeros(np.broadcast(x, y).shape)
        for k1, k2, A in self.modes:
            s = s + A * k2 * math.pi * np.sin(k1 * math.pi * x) * np.cos(k2 * math.pi * y)
        return s

    def f(self, x, y):
        x = np.asarray(x, float); y = np.asarray(y, float)
        s = np.zeros(np.broadcast(x, y).shape)
        for k1, k2, A in self.modes:
            w1, w2 = k1 * math.pi, k2 * math.pi
            sx, cx = np.sin(w1 * x), np.cos(w1 * x)
            sy, cy = np.sin(w2 * y), np.cos(w2 * y)
            s = s + A * (-self.a * w1 * w1 * sx * sy + self.b * w1 * w2 * cx * cy
                         - self.c * w2 * w2 * sx * sy)
        return s


class SinCos:
    """u = sin(p x) cos(q y), the unit-square test of Section 6.1 (p=4, q=3)."""

    def __init__(self, p, q, a, b, c):
        self.p, self.q = float(p), float(q)
        self.a, self.b, self.c = float(a), float(b), float(c)

    def u(self, x, y):
        return np.sin(self.p * np.asarray(x, float)) * np.cos(self.q * np.asarray(y, float))

    def ux(self, x, y):
        return self.p * np.cos(self.p * np.asarray(x, float)) * np.cos(self.q * np.asarray(y, float))

    def uy(self, x, y):
        return -self.q * np.sin(self.p * np.asarray(x, float)) * np.sin(self.q * np.asarray(y, float))

    def f(self, x, y):
        x = np.asarray(x, float); y = np.asarray(y, float)
        p, q = self.p, self.q
        return (-self.a * p * p * np.sin(p * x) * np.cos(q * y)
                - self.b * p * q * np.cos(p * x) * np.sin(q * y)
                - self.c * q * q * np.sin(p * x) * np.cos(q * y))


class Poly:
    """u = sum c_(i,j) x^i y^j, used for exactness checks (degree <= 4)."""

    def __init__(self, coeffs, a, b, c):
        self.coeffs = {(int(i), int(j)): float(v) for (i, j), v in coeffs.items()}
        self.a, self.b, self.c = float(a), float(b), float(c)

    def _eval(self, terms, x, y):
        x = np.asarray(x, float); y = np.asarray(y, float)
        s = np.zeros(np.broadcast(x, y).shape)
        for (i, j), v in terms.items():
            if v != 0.0 and i >= 0 and j >= 0:
                s = s + v * x ** i * y ** j
        return s

    def u(self, x, y):
        return self._eval(self.coeffs, x, y)

    def ux(self, x, y):
        return self._eval({(i - 1, j): v * i for (i, j), v in self.coeffs.items()}, x, y)

    def uy(self, x, y):
        return self._eval({(i, j - 1): v * j for (i, j), v in self.coeffs.items()}, x, y)

    def f(self, x, y):
        t = {}
        for (i, j), v in self.coeffs.items():
            for key, w in (((i - 2, j), self.a * i * (i - 1)), ((i - 1, j - 1), self.b * i * j),
                           ((i, j - 2), self.c * j * (j - 1))):
                t[key] = t.get(key, 0.0) + v * w
        return self._eval(t, x, y)


# ----------------------------------------------------------------------------
# curves
# ----------------------------------------------------------------------------
def box_curve(x0, y0, x1, y1, bc=BC_DIRICHLET, alpha1=1.0, alpha2=0.0):
    """Counter-clockwise box; one segment per side (bottom, right, top, left)."""
    s = lambda p: Segment("line", p, bc, alpha1, alpha2)
    return [s((x0, y0, x1, y0)), s((x1, y0, x1, y1)), s((x1, y1, x0, y1)), s((x0, y1, x0, y0))]


def disk_hole(cx, cy, r, bc=BC_DIRICHLET, alpha1=1.0, alpha2=0.0, theta0=0.3):
    """A circular hole traversed clockwise (Omega outside the disk on the left).
    theta0 places the curve's start point off the grid lines."""
    return [Segment("arc", (cx, cy, r, theta0, theta0 - 2.0 * math.pi), bc, alpha1, alpha2)]


def star_hole(cx, cy, R, r_in, phi, npts=8, bc=BC_ROBIN, alpha1=1.0, alpha2=0.5, round_tips=True):
    """Star polygon with npts tips at radius R and npts valleys at radius r_in
    whose vertices are replaced by circular arcs centred at (cx, cy), each
    joining the points one quarter of the way from the vertex along its two
    adjacent edges; the curve is then made of 2*npts line segments and 2*npts
    arcs meeting at kinks (tangent discontinuities).  With round_tips=False
    only the valleys are rounded and the tips stay sharp corners.
    Returned clockwise (Omega, the outside of the star, on the left)."""
    n = 2 * npts
    ang = [phi + k * math.pi / npts for k in range(n)]
    vert = [(cx + (R if k % 2 == 0 else r_in) * math.cos(ang[k]),
             cy + (R if k % 2 == 0 else r_in) * math.sin(ang[k])) for k in range(n)]
    rounded = [round_tips or k % 2 == 1 for k in range(n)]

    def quarter(V, W):
        return (V[0] + 0.25 * (W[0] - V[0]), V[1] + 0.25 * (W[1] - V[1]))

    def arc(A, B, ccw_turn):
        ta = math.atan2(A[1] - cy, A[0] - cx)
        tb = math.atan2(B[1] - cy, B[0] - cx)
        while tb <= ta:
            tb += 2.0 * math.pi
        while tb - ta > 2.0 * math.pi:
            tb -= 2.0 * math.pi
        return ("arc", (cx, cy, math.hypot(A[0] - cx, A[1] - cy), ta, tb))

    # start/end point of the straight part of edge k -> k+1
    ccw = []
    for k in range(n):
        V0, V1 = vert[k], vert[(k + 1) % n]
        P0 = quarter(V0, V1) if rounded[k] else V0
        P1 = quarter(V1, V0) if rounded[(k + 1) % n] else V1
        ccw.append(("line", (P0[0], P0[1], P1[0], P1[1])))
        if rounded[(k + 1) % n]:
            V2 = vert[(k + 2) % n]
            ccw.append(arc(P1, quarter(V1, V2), True))
    cw = []
    for kind, p in reversed(ccw):
        if kind == "line":
            cw.append(Segment("line", (p[2], p[3], p[0], p[1]), bc, alpha1, alpha2))
        else:
            cw.append(Segment("arc", (p[0], p[1], p[2], p[4], p[3]), bc, alpha1, alpha2))
    return cw


def periodic_config(seed=0, n=64):
    """[0,1]^2 minus a seeded disk, periodic in x (left and right sides),
    Dirichlet at the bottom and the top, Dirichlet on the disk; (a, b, c) =
    (1, 0.5, 2); 4 sine modes sin(k1 pi x) sin(k2 pi y) with even k1, so
    that u is 1-periodic in x."""
    rng = np.random.default_rng([int(seed), 31])
    r = float(rng.uniform(0.1, 0.2))
    cx, cy = (float(v) for v in rng.uniform(0.3, 0.7, size=2))
    ks = rng.integers(1, 5, size=(4, 2))
    amps = rng.uniform(-1.0, 1.0, size=4)
    modes = [(2 * int(1 + ks[m, 0] % 2), int(ks[m, 1]), float(amps[m])) for m in range(4)]
    box = box_curve(0.0, 0.0, 1.0, 1.0)
    box = [Segment(sg.kind, sg.p, BC_PERIODIC if k in (1, 3) else BC_DIRICHLET, 1.0, 0.0)
           for k, sg in enumerate(box)]
    curves = [box, disk_hole(cx, cy, r)]
    return Problem("periodic%d_seed%d" % (n, seed), Grid(0.0, 0.0, 1.0 / n, n, n), curves, 1.0, 0.5, 2.0,
                   SineModes(modes, 1.0, 0.5, 2.0), eps=0.08, meta={"modes": modes})


def bezier_hole(cx, cy, rx, ry, phi=0.0, wobble=(0.0, 0.0, 0.0, 0.0), bc=BC_DIRICHLET, alpha1=1.0, alpha2=0.0):
    """A smooth closed hole made of four cubic Bezier pieces, traversed
    clockwise: an ellipse-like curve with semi-axes (rx, ry) rotated by phi,
    whose four on-curve points move radially by the factors (1 + wobble[k])
    (the tangent handles follow, so the curve stays C1)."""
    kappa = 0.5522847498307936            # handle length of the usual quarter-circle Bezier
    pts = []
    for k in range(4):                     # on-curve points at angles 0, -90, -180, -270 (clockwise)
        th = -0.5 * math.pi * k
        f = 1.0 + wobble[k]
        ex, ey = rx * f * math.cos(th), ry * f * math.sin(th)
        tx, ty = rx * f * math.sin(th), -ry * f * math.cos(th)      # clockwise tangent
        rot = lambda x, y: (cx + x * math.cos(phi) - y * math.sin(phi), cy + x * math.sin(phi) + y * math.cos(phi))
        pts.append((rot(ex, ey), rot(ex + kappa * tx, ey + kappa * ty), rot(ex - kappa * tx, ey - kappa * ty)))
    segs = []
    for k in range(4):
        P0, H0, _ = pts[k]
        P3, _, H3 = pts[(k + 1) % 4]
        segs.append(Segment("cubic", (P0[0], P0[1], H0[0], H0[1], H3[0], H3[1], P3[0], P3[1]), bc, alpha1, alpha2))
    return segs


def bezier_config(seed=0, n=128):
    """[0,1]^2 minus a seeded smooth hole of four cubic Bezier pieces (the
    spline boundaries of Section 2), Neumann on the hole, Dirichlet box;
    (a, b, c) = (1, 0.5, 2); 6 sine modes."""
    rng = np.random.default_rng(seed)
    rx, ry = (float(v) for v in rng.uniform(0.15, 0.25, size=2))
    phi = float(rng.uniform(0.0, math.pi))
    wob = tuple(float(v) for v in rng.uniform(-0.15, 0.15, size=4))
    cx, cy = (float(v) for v in 0.5 + rng.uniform(-0.05, 0.05, size=2))
    modes = _modes(rng, 6)
    curves = [box_curve(0.0, 0.0, 1.0, 1.0), bezier_hole(cx, cy, rx, ry, phi, wob, BC_NEUMANN)]
    return Problem("bezier%d_seed%d" % (n, seed), Grid(0.0, 0.0, 1.0 / n, n, n), curves, 1.0, 0.5, 2.0,
                   SineModes(modes, 1.0, 0.5, 2.0), eps=0.08)


def _modes(rng, count):
    ks = rng.integers(1, 5, size=(count, 2))
    amps = rng.uniform(-1.0, 1.0, size=count)
    return [(int(ks[m, 0]), int(ks[m, 1]), float(amps[m])) for m in range(count)]


def _disks(rng, count, rmin=0.05, rmax=0.15, gap=0.08, lo=0.0, hi=1.0):
    disks = []
    while len(disks) < count:
        r = float(rng.uniform(rmin, rmax))
        cx, cy = (float(v) for v in rng.uniform(lo + r + gap, hi - r - gap, size=2))
        if all(math.hypot(cx - d[0], cy - d[1]) >= r + d[2] + gap for d in disks):
            disks.append((cx, cy, r))
    return disks


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------
def unit_disk_config(seed=0, n=64):
    """Poisson on [0,1]^2 minus the disk of radius 0.2 centred at (0.5,0.5),
    Dirichlet everywhere, 4 seeded sine modes."""
    rng = np.random.default_rng(seed)
    modes = _modes(rng, 4)
    a, b, c = 1.0, 0.0, 1.0
    curves = [box_curve(0.0, 0.0, 1.0, 1.0), disk_hole(0.5, 0.5, 0.2)]
    return Problem("disk64", Grid(0.0, 0.0, 1.0 / n, n, n), curves, a, b, c,
                   SineModes(modes, a, b, c), eps=0.08, meta={"seed": seed, "modes": modes})


def three_disks_config(seed=0, n=1024):
    """[0,1]^2 minus 3 seeded disks (radius U[0.05,0.15]); a=1, b=0.5, c=2;
    Dirichlet outside, Neumann on the holes; 6 seeded sine modes."""
    rng = np.random.default_rng(seed)
    disks = _disks(rng, 3)
    modes = _modes(rng, 6)
    a, b, c = 1.0, 0.5, 2.0
    curves = [box_curve(0.0, 0.0, 1.0, 1.0)] + [disk_hole(x, y, r, BC_NEUMANN) for x, y, r in disks]
    return Problem("three_disks%d" % n, Grid(0.0, 0.0, 1.0 / n, n, n), curves, a, b, c,
                   SineModes(modes, a, b, c), eps=0.08,
                   meta={"seed": seed, "modes": modes, "disks": disks})


def star_config(seed=0, n=4096):
    """[0,1]^2 minus a seeded 8-point star whose valleys are circular arcs and
    whose 8 tips stay sharp corners; a=2, b=-1, c=1; Robin (1, 0.5) on the
    star, Dirichlet outside; 8 seeded sine modes."""
    rng = np.random.default_rng(seed)
    cx, cy = (0.5 + float(v) for v in rng.uniform(-0.03, 0.03, size=2))
    phi = float(rng.uniform(0.0, math.pi / 4))
    R = float(rng.uniform(0.28, 0.32))
    r_in = float(rng.uniform(0.14, 0.18))
    modes = _modes(rng, 8)
    a, b, c = 2.0, -1.0, 1.0
    curves = [box_curve(0.0, 0.0, 1.0, 1.0), star_hole(cx, cy, R, r_in, phi, round_tips=False)]
    return Problem("star%d" % n, Grid(0.0, 0.0, 1.0 / n, n, n), curves, a, b, c,
                   SineModes(modes, a, b, c), eps=0.08,
                   meta={"seed": seed, "modes": modes, "star": (cx, cy, R, r_in, phi)})


def unit_square_config(n=64, a=1.0, b=0.0, c=2.0, bc=BC_DIRICHLET):
    """The unit-square test of Section 6.1: u = sin(4x) cos(3y), (a,b,c)=(1,0,2)."""
    curves = [box_curve(0.0, 0.0, 1.0, 1.0, bc)]
    return Problem("unit_square%d" % n, Grid(0.0, 0.0, 1.0 / n, n, n), curves, a, b, c,
                   SinCos(4.0, 3.0, a, b, c), eps=0.1)


def serving_request(trace_seed, request_id):
    """One request of the serving trace: grid uniform over {128..2048}^2,
    1-5 disk holes with mixed boundary conditions, a, c ~ U[0.5, 2],
    |b| < sqrt(ac), 4-8 sine modes."""
    rng = np.random.default_rng([int(trace_seed), int(request_id)])
    n = int(rng.choice([128, 256, 512, 1024, 2048]))
    nholes = int(rng.integers(1, 6))
    disks = _disks(rng, nholes)
    bcs = [str(rng.choice([BC_DIRICHLET, BC_NEUMANN, BC_ROBIN])) for _ in range(nholes)]
    a = float(rng.uniform(0.5, 2.0)); c = float(rng.uniform(0.5, 2.0))
    b = float(rng.uniform(-1.0, 1.0)) * math.sqrt(a * c) * 0.95
    modes = _modes(rng, int(rng.integers(4, 9)))
    curves = [box_curve(0.0, 0.0, 1.0, 1.0)]
    for (x, y, r), bc in zip(disks, bcs):
        curves.append(disk_hole(x, y, r, bc, 1.0, 0.5))
    return Problem("req%d_%d" % (trace_seed, request_id), Grid(0.0, 0.0, 1.0 / n, n, n), curves,
                   a, b, c, SineModes(modes, a, b, c), eps=0.08,
                   meta={"disks": disks, "bcs": bcs, "modes": modes})


def with_grid(problem, n):
    """The same problem on an n x n grid of the same box."""
    g = problem.grid
    L = g.h * g.nx
    return Problem(problem.name, Grid(g.x0, g.y0, L / n, n, n), problem.curves, problem.a,
                   problem.b, problem.c, problem.solution, problem.eps, dict(problem.meta))


def serving_geometry(seed, n=2048):
    """One geometry of the resident-serving workload: a seeded star (its
    boundary condition uniform over N, R) on even seeds, 1-5 seeded disks
    with mixed boundary conditions on odd seeds; a, c ~ U[0.5, 2],
    |b| < sqrt(ac); n x n cells.  (A Dirichlet star is left out: the V-cycle
    diverges on it, in the oracle as on the GPU.)"""
    rng = np.random.default_rng([int(seed), 4099])
    a = float(rng.uniform(0.5, 2.0)); c = float(rng.uniform(0.5, 2.0))
    b = float(rng.uniform(-1.0, 1.0)) * math.sqrt(a * c) * 0.95
    curves = [box_curve(0.0, 0.0, 1.0, 1.0)]
    if seed % 2 == 0:
        cx, cy = (0.5 + float(v) for v in rng.uniform(-0.03, 0.03, size=2))
        phi = float(rng.uniform(0.0, math.pi / 4))
        R = float(rng.uniform(0.28, 0.32)); r_in = float(rng.uniform(0.14, 0.18))
        bc = str(rng.choice([BC_NEUMANN, BC_ROBIN]))
        curves.append(star_hole(cx, cy, R, r_in, phi, bc=bc, alpha1=1.0, alpha2=0.5, round_tips=False))
    else:
        for (x, y, r) in _disks(rng, int(rng.integers(1, 6))):
            bc = str(rng.choice([BC_DIRICHLET, BC_NEUMANN, BC_ROBIN]))
            curves.append(disk_hole(x, y, r, bc, 1.0, 0.5))
    modes = _modes(rng, 6)
    return Problem("geom%d_%d" % (seed, n), Grid(0.0, 0.0, 1.0 / n, n, n), curves, a, b, c,
                   SineModes(modes, a, b, c), eps=0.08)


def with_solution(problem, seed, count=6):
    """The same geometry and operator with another seeded sine-mode solution
    (another right-hand side)."""
    rng = np.random.default_rng([int(seed), 7919])
    modes = _modes(rng, count)
    meta = dict(problem.meta)
    meta["modes"] = modes
    return Problem(problem.name, problem.grid, problem.curves, problem.a, problem.b, problem.c,
                   SineModes(modes, problem.a, problem.b, problem.c), problem.eps, meta)

