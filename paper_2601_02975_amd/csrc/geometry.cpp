// Cut cells and cell merging (Section 3, Algorithm 1), host side.
//
// Holes are closed curves of lines and arcs; the outer boundary is the grid
// box.  Each hole is cut at its crossings with the grid lines into pieces,
// each inside one grid cell; consecutive pieces in a cell form a "run" that
// enters and leaves the cell through its perimeter.  Walking the perimeter
// counter-clockwise from the exit of a run reaches the entry of the next run
// of the same component, so runs and perimeter pieces close into loops, one
// per connected component.  Moments follow from Green's theorem
//   ∬ X^p Y^q dX dY = ∮ X^(p+1)/(p+1) Y^q dY
// in coordinates scaled about the cell centre.
#include <algorithm>
#include <cmath>
#include <functional>
#include <map>

#include "mg_internal.hpp"

namespace mgc {

const int MONO_P[NB] = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0, 4, 3, 2, 1, 0};
const int MONO_Q[NB] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3, 0, 1, 2, 3, 4};

int mono_index(int p, int q) {
    int d = p + q;
    return d * (d + 1) / 2 + (d - p);
}

void Seg::point(double t, double &x, double &y) const {
    if (kind == MG_SEG_LINE) {
        x = p[0] + t * (p[2] - p[0]);
        y = p[1] + t * (p[3] - p[1]);
    } else if (kind == MG_SEG_CUBIC) {
        const double u = 1.0 - t, b0 = u * u * u, b1 = 3.0 * u * u * t, b2 = 3.0 * u * t * t, b3 = t * t * t;
        x = b0 * p[0] + b1 * p[2] + b2 * p[4] + b3 * p[6];
        y = b0 * p[1] + b1 * p[3] + b2 * p[5] + b3 * p[7];
    } else {
        double th = p[3] + t * (p[4] - p[3]);
        x = p[0] + p[2] * std::cos(th);
        y = p[1] + p[2] * std::sin(th);
    }
}

void Seg::deriv(double t, double &dx, double &dy) const {
    if (kind == MG_SEG_LINE) {
        dx = p[2] - p[0];
        dy = p[3] - p[1];
    } else if (kind == MG_SEG_CUBIC) {
        const double u = 1.0 - t, d0 = 3.0 * u * u, d1 = 6.0 * u * t, d2 = 3.0 * t * t;
        dx = d0 * (p[2] - p[0]) + d1 * (p[4] - p[2]) + d2 * (p[6] - p[4]);
        dy = d0 * (p[3] - p[1]) + d1 * (p[5] - p[3]) + d2 * (p[7] - p[5]);
    } else {
        double sw = p[4] - p[3];
        double th = p[3] + t * sw;
        dx = -p[2] * sw * std::sin(th);
        dy = p[2] * sw * std::cos(th);
    }
}

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

void full_moments(double mom[NB]) {
    for (int k = 0; k < NB; ++k) {
        int a = MONO_P[k], b = MONO_Q[k];
        double ia = (a % 2) ? 0.0 : 1.0 / ((a + 1) * std::pow(2.0, a));
        double ib = (b % 2) ? 0.0 : 1.0 / ((b + 1) * std::pow(2.0, b));
        mom[k] = ia * ib;
    }
}

static double binom(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

// ∬ (X + dx)^a (Y + dy)^b from the moments ∬ X^p Y^q
void shift_moments(const double *m, int dx, int dy, double *out) {
    for (int k = 0; k < NB; ++k) {
        int a = MONO_P[k], b = MONO_Q[k];
        double s = 0.0;
        for (int p = 0; p <= a; ++p)
            for (int q = 0; q <= b; ++q)
                s += binom(a, p) * binom(b, q) * std::pow((double)dx, a - p) * std::pow((double)dy, b - q) *
                     m[mono_index(p, q)];
        out[k] = s;
    }
}

namespace {

struct GL {
    std::vector<double> x4, w4, x16, w16;
    GL() {
        gauss_legendre(4, x4, w4);
        gauss_legendre(16, x16, w16);
    }
};
const GL &gl() {
    static GL g;
    return g;
}

// real roots of c3 t^3 + c2 t^2 + c1 t + c0 (leading zeros allowed): the
// closed forms (trigonometric for three real roots), each polished by
// Newton steps on the original polynomial
void real_roots(double c3, double c2, double c1, double c0, double scale, std::vector<double> &r) {
    r.clear();
    if (std::fabs(c3) <= 1e-14 * scale) {
        if (std::fabs(c2) <= 1e-14 * scale) {
            if (std::fabs(c1) > 1e-14 * scale) r.push_back(-c0 / c1);
            return;
        }
        const double disc = c1 * c1 - 4.0 * c2 * c0;
        if (disc < 0.0) {
            if (disc > -1e-24 * scale * scale) r.push_back(-c1 / (2.0 * c2));
            return;
        }
        const double q = -0.5 * (c1 + std::copysign(std::sqrt(disc), c1));
        r.push_back(q / c2);
        if (q != 0.0) r.push_back(c0 / q);
    } else {
        const double a = c2 / c3, b = c1 / c3, c = c0 / c3;
        const double Q = (a * a - 3.0 * b) / 9.0, R = (2.0 * a * a * a - 9.0 * a * b + 27.0 * c) / 54.0;
        if (R * R < Q * Q * Q) {
            const double th = std::acos(std::max(-1.0, std::min(1.0, R / std::sqrt(Q * Q * Q))));
            const double m = -2.0 * std::sqrt(Q);
            for (int k = 0; k < 3; ++k) r.push_back(m * std::cos((th + 2.0 * M_PI * (k - 1)) / 3.0) - a / 3.0);
        } else {
            const double A = -std::copysign(std::cbrt(std::fabs(R) + std::sqrt(R * R - Q * Q * Q)), R);
            const double B = A != 0.0 ? Q / A : 0.0;
            r.push_back(A + B - a / 3.0);
        }
    }
    for (double &t : r)
        for (int it = 0; it < 4; ++it) {
            const double f = ((c3 * t + c2) * t + c1) * t + c0, d = (3.0 * c3 * t + 2.0 * c2) * t + c1;
            if (d == 0.0) break;
            t -= f / d;
        }
}

// parameters t in (0,1) where coordinate `coord` of seg equals value
void line_params(const Seg &s, int coord, double value, std::vector<double> &out) {
    if (s.kind == MG_SEG_CUBIC) {
        const double q0 = s.p[coord], q1 = s.p[2 + coord], q2 = s.p[4 + coord], q3 = s.p[6 + coord];
        const double c3 = -q0 + 3.0 * q1 - 3.0 * q2 + q3, c2 = 3.0 * q0 - 6.0 * q1 + 3.0 * q2;
        const double c1 = -3.0 * q0 + 3.0 * q1, c0 = q0 - value;
        const double scale = std::max(std::max(std::fabs(q0), std::fabs(q1)), std::max(std::fabs(q2), std::fabs(q3))) +
                             std::fabs(value);
        if (std::fabs(c3) <= 1e-14 * scale && std::fabs(c2) <= 1e-14 * scale && std::fabs(c1) <= 1e-14 * scale) {
            if (std::fabs(c0) <= 1e-14 * scale) fail(MG_ERR_GEOMETRY, "segment lies on a grid line");
            return;
        }
        std::vector<double> r;
        real_roots(c3, c2, c1, c0, scale, r);
        std::sort(r.begin(), r.end());
        size_t first = out.size();
        for (double t : r) {
            if (!(t > -1e-15 && t < 1.0 + 1e-15)) continue;
            const double d = (3.0 * c3 * t + 2.0 * c2) * t + c1;
            if (std::fabs(d) < 1e-9 * scale) fail(MG_ERR_GEOMETRY, "cubic segment tangent to a grid line");
            bool dup = false;
            for (size_t k = first; k < out.size(); ++k) dup = dup || std::fabs(out[k] - t) < 1e-13;
            if (!dup) out.push_back(t);
        }
        return;
    }
    if (s.kind == MG_SEG_LINE) {
        double a = coord == 0 ? s.p[0] : s.p[1];
        double b = coord == 0 ? s.p[2] : s.p[3];
        if (a == b) {
            if (a == value) fail(MG_ERR_GEOMETRY, "segment lies on a grid line");
            return;
        }
        double t = (value - a) / (b - a);
        if (t > -1e-15 && t < 1.0 + 1e-15) out.push_back(t);
        return;
    }
    double cc = coord == 0 ? s.p[0] : s.p[1];
    double r = s.p[2], t0 = s.p[3], t1 = s.p[4];
    double q = (value - cc) / r;
    if (std::fabs(q) > 1.0) return;
    if (std::fabs(std::fabs(q) - 1.0) < 1e-12) fail(MG_ERR_GEOMETRY, "arc tangent to a grid line");
    double base = coord == 0 ? std::acos(q) : std::asin(q);
    double cands[2] = {base, coord == 0 ? -base : M_PI - base};
    double lo = std::min(t0, t1), hi = std::max(t0, t1);
    for (double th : cands) {
        long k0 = (long)std::floor((lo - th) / (2.0 * M_PI)) - 1;
        for (long k = k0; k < k0 + 4; ++k) {
            double tt = th + 2.0 * M_PI * k;
            if (tt > lo - 1e-15 && tt < hi + 1e-15) out.push_back((tt - t0) / (t1 - t0));
        }
    }
}

int64_t face_key(int i, int j, int side) {
    // vertical face at x-line k between cells (k-1, j) and (k, j): kind 0
    // horizontal face at y-line l between cells (i, l-1) and (i, l): kind 1
    int kind, a, b;
    if (side == 0) { kind = 1; a = i; b = j; }
    else if (side == 1) { kind = 0; a = i + 1; b = j; }
    else if (side == 2) { kind = 1; a = i; b = j + 1; }
    else { kind = 0; a = i; b = j; }
    return ((int64_t)kind << 62) | ((int64_t)a << 31) | (int64_t)b;
}

struct Crossing { double t; int kind; int line; };   // kind 0: x = const line, 1: y = const

struct Piece {
    int seg;
    double ta, tb;
    bool has_start, has_end;
    Crossing cs, ce;
};

struct Run {
    int ci, cj;
    std::vector<BPiece> pieces;
    double entry = -1, exit = -1;
};

double tau_of(const mg_grid &g, int i, int j, const Seg &s, double t, const Crossing &c) {
    double x, y;
    s.point(t, x, y);
    double X0 = g.x0 + i * g.h, Y0 = g.y0 + j * g.h;
    if (c.kind == 1) {
        if (c.line == j) return (x - X0) / g.h;
        if (c.line == j + 1) return 2.0 + (X0 + g.h - x) / g.h;
    } else {
        if (c.line == i + 1) return 1.0 + (y - Y0) / g.h;
        if (c.line == i) return 3.0 + (Y0 + g.h - y) / g.h;
    }
    fail(MG_ERR_GEOMETRY, "crossing not on the cell perimeter");
}

double mod4(double x) { return x - 4.0 * std::floor(x / 4.0); }

void curve_moments(const Seg &s, double ta, double tb, double xc, double yc, double h, double *mom) {
    const GL &G = gl();
    const std::vector<double> &X = s.kind == MG_SEG_LINE ? G.x4 : G.x16;
    const std::vector<double> &W = s.kind == MG_SEG_LINE ? G.w4 : G.w16;
    for (size_t n = 0; n < X.size(); ++n) {
        double t = 0.5 * (tb - ta) * X[n] + 0.5 * (ta + tb);
        double wt = 0.5 * (tb - ta) * W[n];
        double x, y, dx, dy;
        s.point(t, x, y);
        s.deriv(t, dx, dy);
        double Xs = (x - xc) / h, Ys = (y - yc) / h, dYs = dy / h;
        for (int k = 0; k < NB; ++k) {
            int a = MONO_P[k], b = MONO_Q[k];
            mom[k] += wt * std::pow(Xs, a + 1) / (a + 1) * std::pow(Ys, b) * dYs;
        }
    }
}

void edge_moments(int side, double s0, double s1, double *mom) {
    double Xv, Ya, Yb;
    if (side == 1) { Xv = 0.5; Ya = s0 - 0.5; Yb = s1 - 0.5; }
    else if (side == 3) { Xv = -0.5; Ya = 0.5 - s0; Yb = 0.5 - s1; }
    else return;
    for (int k = 0; k < NB; ++k) {
        int a = MONO_P[k], b = MONO_Q[k];
        mom[k] += std::pow(Xv, a + 1) / (a + 1) * (std::pow(Yb, b + 1) - std::pow(Ya, b + 1)) / (b + 1);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
void build_cutgrid(const Curves &cv, const mg_grid &g, double eps, CutGrid &cg) {
    const int nx = g.nx, ny = g.ny;
    const double h = g.h;
    cg.g = g;
    cg.eps = eps;
    // outer box: bottom, right, top, left
    {
        const auto &box = cv.c.at(0);
        double x1 = g.x0 + nx * h, y1 = g.y0 + ny * h;
        double want[4][4] = {{g.x0, g.y0, x1, g.y0}, {x1, g.y0, x1, y1}, {x1, y1, g.x0, y1}, {g.x0, y1, g.x0, g.y0}};
        if (box.size() != 4) fail(MG_ERR_GEOMETRY, "the outer curve must be the grid box");
        for (int s = 0; s < 4; ++s) {
            if (box[s].kind != MG_SEG_LINE) fail(MG_ERR_GEOMETRY, "the outer curve must be the grid box");
            for (int k = 0; k < 4; ++k)
                if (std::fabs(box[s].p[k] - want[s][k]) > 1e-12 * std::max(1.0, std::fabs(want[s][k])))
                    fail(MG_ERR_GEOMETRY, "the outer curve must be the counter-clockwise grid box");
            cg.box_bc[s] = box[s].bc;
            cg.box_al[s][0] = box[s].al1;
            cg.box_al[s][1] = box[s].al2;
        }
        for (int s = 0; s < 2; ++s)
            if ((box[s].bc == MG_BC_PERIODIC) != (box[s + 2].bc == MG_BC_PERIODIC))
                fail(MG_ERR_GEOMETRY, "periodic box sides must come in opposite pairs");
        for (size_t k = 1; k < cv.c.size(); ++k)
            for (const Seg &sg : cv.c[k])
                if (sg.bc == MG_BC_PERIODIC) fail(MG_ERR_GEOMETRY, "periodic conditions apply to box sides only");
    }
    // runs per cell
    std::map<int, std::vector<Run>> runs;
    for (size_t ci = 1; ci < cv.c.size(); ++ci) {
        const auto &curve = cv.c[ci];
        std::vector<Piece> pieces;
        size_t ncross = 0;
        for (size_t si = 0; si < curve.size(); ++si) {
            const Seg &s = curve[si];
            double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
            for (int k = 0; k <= 64; ++k) {
                double x, y;
                s.point(k / 64.0, x, y);
                xmin = std::min(xmin, x); xmax = std::max(xmax, x);
                ymin = std::min(ymin, y); ymax = std::max(ymax, y);
            }
            if (s.kind == MG_SEG_CUBIC)            // the control polygon bounds the curve
                for (int k = 0; k < 4; ++k) {
                    xmin = std::min(xmin, s.p[2 * k]); xmax = std::max(xmax, s.p[2 * k]);
                    ymin = std::min(ymin, s.p[2 * k + 1]); ymax = std::max(ymax, s.p[2 * k + 1]);
                }
            int kx0 = std::max(0, (int)std::floor((xmin - g.x0) / h) - 1);
            int kx1 = std::min(nx, (int)std::ceil((xmax - g.x0) / h) + 1);
            int ky0 = std::max(0, (int)std::floor((ymin - g.y0) / h) - 1);
            int ky1 = std::min(ny, (int)std::ceil((ymax - g.y0) / h) + 1);
            std::vector<Crossing> cr;
            std::vector<double> ts;
            for (int k = kx0; k <= kx1; ++k) {
                ts.clear();
                line_params(s, 0, g.x0 + k * h, ts);
                for (double t : ts) cr.push_back({t, 0, k});
            }
            for (int l = ky0; l <= ky1; ++l) {
                ts.clear();
                line_params(s, 1, g.y0 + l * h, ts);
                for (double t : ts) cr.push_back({t, 1, l});
            }
            std::sort(cr.begin(), cr.end(), [](const Crossing &a, const Crossing &b) { return a.t < b.t; });
            for (auto &c : cr)
                if (c.t < 1e-12 || c.t > 1.0 - 1e-12) fail(MG_ERR_GEOMETRY, "curve vertex on a grid line");
            for (size_t k = 0; k + 1 < cr.size(); ++k)
                if (cr[k + 1].t - cr[k].t < 1e-12) fail(MG_ERR_GEOMETRY, "curve passes through a grid vertex");
            ncross += cr.size();
            double prev_t = 0.0;
            bool prev_has = false;
            Crossing prev_c{};
            for (size_t k = 0; k <= cr.size(); ++k) {
                Piece p;
                p.seg = (int)si;
                p.ta = prev_t;
                p.has_start = prev_has;
                p.cs = prev_c;
                if (k < cr.size()) {
                    p.tb = cr[k].t;
                    p.has_end = true;
                    p.ce = cr[k];
                } else {
                    p.tb = 1.0;
                    p.has_end = false;
                }
                pieces.push_back(p);
                if (k < cr.size()) {
                    prev_t = cr[k].t;
                    prev_has = true;
                    prev_c = cr[k];
                }
            }
        }
        if (ncross == 0) fail(MG_ERR_GEOMETRY, "a hole lies inside a single cell");
        size_t start = 0;
        while (!pieces[start].has_start) ++start;
        Run *cur = nullptr;
        for (size_t k = 0; k < pieces.size(); ++k) {
            const Piece &p = pieces[(start + k) % pieces.size()];
            const Seg &s = curve[p.seg];
            if (p.has_start) {
                double xm, ym;
                s.point(0.5 * (p.ta + p.tb), xm, ym);
                int i = (int)std::floor((xm - g.x0) / h), j = (int)std::floor((ym - g.y0) / h);
                if (i < 0 || i >= nx || j < 0 || j >= ny) fail(MG_ERR_GEOMETRY, "hole leaves the box");
                auto &lst = runs[j * nx + i];
                lst.emplace_back();
                cur = &lst.back();
                cur->ci = i;
                cur->cj = j;
                cur->entry = tau_of(g, i, j, s, p.ta, p.cs);
            }
            cur->pieces.push_back({(int)ci, p.seg, p.ta, p.tb});
            if (p.has_end) cur->exit = tau_of(g, cur->ci, cur->cj, s, p.tb, p.ce);
        }
    }

    // cells whose centre lies in Omega (crossing parity along centre lines)
    std::vector<uint8_t> inside((size_t)nx * ny, 1);
    {
        std::vector<double> xs, ts;
        for (int j = 0; j < ny; ++j) {
            double yc = g.y0 + (j + 0.5) * h;
            for (size_t ci = 1; ci < cv.c.size(); ++ci) {
                xs.clear();
                for (const Seg &s : cv.c[ci]) {
                    ts.clear();
                    line_params(s, 1, yc, ts);
                    for (double t : ts)
                        if (t >= 0.0 && t < 1.0) {
                            double x, y;
                            s.point(t, x, y);
                            xs.push_back(x);
                        }
                }
                if (xs.empty()) continue;
                std::sort(xs.begin(), xs.end());
                for (int i = 0; i < nx; ++i) {
                    double xc = g.x0 + (i + 0.5) * h;
                    size_t right = xs.end() - std::upper_bound(xs.begin(), xs.end(), xc);
                    if (right % 2) inside[(size_t)j * nx + i] = 0;
                }
            }
        }
    }

    // components of cut cells
    std::vector<Comp> &comps = cg.comps;
    comps.clear();
    std::map<int, std::vector<int>> cellcomps;           // cut cell -> component ids (ordered)
    for (auto &kv : runs) {
        int cell = kv.first;
        auto &rl = kv.second;
        int i = cell % nx, j = cell / nx;
        std::vector<int> order(rl.size());
        for (size_t k = 0; k < rl.size(); ++k) order[k] = (int)k;
        std::sort(order.begin(), order.end(), [&](int a, int b) { return rl[a].entry < rl[b].entry; });
        std::vector<int> nxt(rl.size());
        for (int r : order) {
            double tout = rl[r].exit;
            int best = -1;
            double bv = 1e300;
            for (int q : order) {
                double v = mod4(rl[q].entry - tout);
                if (v < bv) { bv = v; best = q; }
            }
            nxt[r] = best;
        }
        std::vector<char> seen(rl.size(), 0);
        std::vector<int> ids;
        double xc = g.x0 + (i + 0.5) * h, yc = g.y0 + (j + 0.5) * h;
        for (int r0 : order) {
            if (seen[r0]) continue;
            Comp c;
            c.ci = i; c.cj = j; c.full = false;
            std::fill(c.mom, c.mom + NB, 0.0);
            c.key = rl[r0].entry;
            int r = r0;
            while (!seen[r]) {
                seen[r] = 1;
                for (auto &bp : rl[r].pieces) {
                    curve_moments(cv.c[bp.curve][bp.seg], bp.ta, bp.tb, xc, yc, h, c.mom);
                    c.bp.push_back(bp);
                    LoopItem it{};
                    it.is_edge = 0;
                    it.piece = bp;
                    c.items.push_back(it);
                }
                double tout = rl[r].exit;
                int q = nxt[r];
                double span = mod4(rl[q].entry - tout);
                double pos = tout, remaining = span;
                while (remaining > 1e-15) {
                    double fl = std::floor(pos + 1e-15);
                    int side = ((int)fl % 4 + 4) % 4;
                    double s0 = pos - fl;
                    if (s0 < 0) s0 = 0.0;
                    double step = std::min(remaining, 1.0 - s0);
                    edge_moments(side, s0, s0 + step, c.mom);
                    LoopItem it{};
                    it.is_edge = 1;
                    it.side = side;
                    it.s0 = s0;
                    it.s1 = s0 + step;
                    c.items.push_back(it);
                    double lo = side <= 1 ? s0 : 1.0 - (s0 + step);
                    double hi = side <= 1 ? s0 + step : 1.0 - s0;
                    c.faces.push_back({face_key(i, j, side), lo, hi});
                    remaining -= step;
                    pos = mod4(pos + step);
                }
                r = q;
            }
            if (c.mom[0] <= 0.0) fail(MG_ERR_GEOMETRY, "negatively oriented loop (hole inside a cell)");
            c.parent = (int)comps.size();
            c.vtot = c.mom[0];
            ids.push_back((int)comps.size());
            comps.push_back(std::move(c));
        }
        std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) { return comps[a].key < comps[b].key; });
        cellcomps[cell] = ids;
        inside[cell] = 0;
    }

    // --- Algorithm 1 ----------------------------------------------------------
    std::map<int, int> fullc;                                 // regular cell -> component id
    auto full_comp = [&](int cell) {
        auto it = fullc.find(cell);
        if (it != fullc.end()) return it->second;
        Comp c;
        c.ci = cell % nx; c.cj = cell / nx; c.full = true;
        full_moments(c.mom);
        for (int s = 0; s < 4; ++s) c.faces.push_back({face_key(c.ci, c.cj, s), 0.0, 1.0});
        c.key = 0.0;
        c.parent = (int)comps.size();
        c.vtot = 1.0;
        comps.push_back(std::move(c));
        fullc[cell] = (int)comps.size() - 1;
        return (int)comps.size() - 1;
    };
    std::function<int(int)> find = [&](int c) {
        while (comps[c].parent != c) {
            comps[c].parent = comps[comps[c].parent].parent;
            c = comps[c].parent;
        }
        return c;
    };
    auto comps_of = [&](int i, int j, std::vector<int> &out) {
        out.clear();
        if (i < 0 || i >= nx || j < 0 || j >= ny) return;
        int cell = j * nx + i;
        auto it = cellcomps.find(cell);
        if (it != cellcomps.end()) { out = it->second; return; }
        if (inside[cell]) out.push_back(full_comp(cell));
    };
    auto touching = [&](int c, int i, int j, std::vector<int> &out) {
        std::vector<int> cand;
        comps_of(i, j, cand);
        out.clear();
        for (int oc : cand) {
            bool hit = false;
            for (auto &f1 : comps[c].faces) {
                for (auto &f2 : comps[oc].faces)
                    if (f1.key == f2.key && std::min(f1.hi, f2.hi) - std::max(f1.lo, f2.lo) > 1e-9) { hit = true; break; }
                if (hit) break;
            }
            if (hit) out.push_back(oc);
        }
    };
    auto absorb = [&](int target, int src) {
        comps[target].absorbed.push_back(src);
        comps[src].parent = target;
        comps[target].vtot += comps[src].vtot;
    };
    const int NBR[4][2] = {{-1, 0}, {1, 0}, {0, -1}, {0, 1}};
    std::vector<int> tmp;
    // lines 2-7: minor components
    for (auto &kv : cellcomps) {
        (void)kv;
    }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            auto it = cellcomps.find(j * nx + i);
            if (it == cellcomps.end() || it->second.size() < 2) continue;
            const auto lst = it->second;
            int m = 0;
            for (size_t k = 1; k < lst.size(); ++k)
                if (comps[lst[k]].mom[0] > comps[lst[m]].mom[0]) m = (int)k;
            for (size_t k = 0; k < lst.size(); ++k) {
                if ((int)k == m) continue;
                int rk = find(lst[k]);
                int best = -1;
                double bestval = 0.0;
                for (auto &d : NBR) {
                    touching(lst[k], i + d[0], j + d[1], tmp);
                    for (int oc : tmp) {
                        int ro = find(oc);
                        if (ro == rk) continue;
                        double val = std::fabs(comps[ro].vtot + comps[rk].vtot - 1.0);
                        if (best < 0 || val < bestval - 1e-12) { best = ro; bestval = val; }
                    }
                }
                if (best < 0) fail(MG_ERR_GEOMETRY, "a minor component has no neighbour to merge into");
                absorb(best, rk);
            }
        }
    // lines 8-11: small cells
    std::map<int, int> mainc;
    for (auto &kv : cellcomps) {
        const auto &lst = kv.second;
        int m = 0;
        for (size_t k = 1; k < lst.size(); ++k)
            if (comps[lst[k]].mom[0] > comps[lst[m]].mom[0]) m = (int)k;
        mainc[kv.first] = lst[m];
    }
    auto cell_root = [&](int cell) {
        auto it = mainc.find(cell);
        if (it != mainc.end()) return find(it->second);
        return find(full_comp(cell));
    };
    std::function<void(int, std::vector<int> &)> members = [&](int root, std::vector<int> &out) {
        out.clear();
        std::vector<int> stack{root};
        while (!stack.empty()) {
            int c = stack.back();
            stack.pop_back();
            out.push_back(c);
            for (int a : comps[c].absorbed) stack.push_back(a);
        }
    };
    std::vector<uint8_t> removed((size_t)nx * ny, 0);
    std::vector<int> mem;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            int cell = j * nx + i;
            if (!mainc.count(cell) || removed[cell]) continue;
            int r = cell_root(cell);
            if (comps[r].ci != i || comps[r].cj != j) fail(MG_ERR_GEOMETRY, "main component absorbed elsewhere");
            if (comps[r].vtot >= eps) continue;
            members(r, mem);
            int best = -1;
            double bestval = 0.0;
            for (auto &d : NBR) {
                int ni = i + d[0], nj = j + d[1];
                if (ni < 0 || ni >= nx || nj < 0 || nj >= ny) continue;
                int nb = nj * nx + ni;
                if (removed[nb]) continue;
                if (!mainc.count(nb) && !inside[nb]) continue;
                int rn = cell_root(nb);
                if (comps[rn].ci != ni || comps[rn].cj != nj) continue;
                bool hit = false;
                for (int c : mem) {
                    for (auto &dd : NBR) {
                        touching(c, comps[c].ci + dd[0], comps[c].cj + dd[1], tmp);
                        for (int oc : tmp)
                            if (find(oc) == rn) { hit = true; break; }
                        if (hit) break;
                    }
                    if (hit) break;
                }
                if (!hit) continue;
                double val = std::fabs(comps[rn].vtot + comps[r].vtot - 1.0);
                if (best < 0 || val < bestval - 1e-12) { best = rn; bestval = val; }
            }
            if (best < 0) fail(MG_ERR_GEOMETRY, "a small cell has no neighbour to merge into");
            absorb(best, r);
            removed[cell] = 1;
        }

    // results
    cg.active.assign((size_t)nx * ny, 0);
    cg.regular = inside;
    for (size_t k = 0; k < inside.size(); ++k) cg.active[k] = inside[k];
    for (auto &kv : cellcomps)
        if (!removed[kv.first]) cg.active[kv.first] = 1;
    cg.irr_slot.assign((size_t)nx * ny, -1);
    cg.irr_cells.clear();
    cg.irr.clear();
    std::vector<int> roots_cells;
    for (auto &kv : mainc)
        if (!removed[kv.first]) roots_cells.push_back(kv.first);
    for (auto &kv : fullc) roots_cells.push_back(kv.first);
    std::sort(roots_cells.begin(), roots_cells.end());
    roots_cells.erase(std::unique(roots_cells.begin(), roots_cells.end()), roots_cells.end());
    for (int cell : roots_cells) {
        int r = cell_root(cell);
        members(r, mem);
        if (mem.size() == 1 && fullc.count(cell) && !mainc.count(cell)) continue;   // untouched regular cell
        int i = cell % nx, j = cell / nx;
        cg.regular[cell] = 0;
        CellData d;
        std::fill(d.mom, d.mom + NB, 0.0);
        double sh[NB];
        for (int c : mem) {
            shift_moments(comps[c].mom, comps[c].ci - i, comps[c].cj - j, sh);
            for (int k = 0; k < NB; ++k) d.mom[k] += sh[k];
            for (auto &bp : comps[c].bp) d.bp.push_back(bp);
        }
        d.members = mem;
        cg.irr_slot[cell] = (int)cg.irr.size();
        cg.irr_cells.push_back(cell);
        cg.irr.push_back(std::move(d));
    }
    cg.owner.assign((size_t)nx * ny, -1);
    for (int cell = 0; cell < nx * ny; ++cell)
        if (removed[cell]) {
            int r = find(mainc[cell]);
            cg.owner[cell] = comps[r].cj * nx + comps[r].ci;
        }
    cg.volfrac.assign((size_t)nx * ny, 0.0);
    for (int cell = 0; cell < nx * ny; ++cell) {
        if (cg.regular[cell]) cg.volfrac[cell] = 1.0;
        else if (cg.irr_slot[cell] >= 0) cg.volfrac[cell] = cg.irr[cg.irr_slot[cell]].mom[0];
    }
}

void cell_moments(const CutGrid &cg, int i, int j, double mom[NB]) {
    int slot = cg.irr_slot[(size_t)j * cg.g.nx + i];
    if (slot >= 0) {
        for (int k = 0; k < NB; ++k) mom[k] = cg.irr[slot].mom[k];
    } else {
        full_moments(mom);
    }
}

}  // namespace mgc
