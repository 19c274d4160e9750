// Exact solve with the PLG block A22 (eq. (5.6)), set up for the GPU.
//
// The PLG cells are ordered along the boundary curves (Definition 5.1): by
// the curve closest to the cell centre, then by the parameter of the closest
// point on it.  In that order A22 is banded apart from O(1) wrap-around
// couplings (Lemma 5.2).  The paper factors it as a bordered band LU
// (Definition 5.3), whose triangular solves are sequential chains of length
// m.  Here the chain of each curve is cut into segments separated by runs of
// "separator" unknowns at least one bandwidth long, so that segments couple
// only through separators; any remaining coupling moves its column into the
// separator set.  With B the segment blocks and S the separators,
//     y = B^{-1} t_B,  x_S = S'^{-1} (t_S - A_SB y),  x_B = y - B^{-1} A_BS x_S,
// where S' = A_SS - A_SB B^{-1} A_BS.  B^{-1} (per segment), B^{-1} A_BS and
// S'^{-1} are dense and precomputed, so a solve is three parallel passes.
#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>

#include "plgsolve.hpp"

namespace mgc {

namespace {

// closest point of a segment to (px, py): returns squared distance and t
void closest_on_seg(const Seg &s, double px, double py, double &d2, double &t) {
    if (s.kind == MG_SEG_CUBIC) {
        // the nearest of 33 samples, refined by Newton steps on
        // (B(t) - p) . B'(t) = 0 within [0, 1]
        double best = 1e300;
        for (int k = 0; k <= 32; ++k) {
            double x, y;
            s.point(k / 32.0, x, y);
            const double d = (x - px) * (x - px) + (y - py) * (y - py);
            if (d < best) { best = d; t = k / 32.0; }
        }
        for (int it = 0; it < 8; ++it) {
            double x, y, dx, dy, x2, y2;
            s.point(t, x, y);
            s.deriv(t, dx, dy);
            const double e = 1e-6;
            s.deriv(std::min(1.0, t + e), x2, y2);
            const double g = (x - px) * dx + (y - py) * dy;
            const double gp = dx * dx + dy * dy + (x - px) * (x2 - dx) / e + (y - py) * (y2 - dy) / e;
            if (gp <= 0.0) break;
            t = std::min(1.0, std::max(0.0, t - g / gp));
        }
        double x, y;
        s.point(t, x, y);
        d2 = (x - px) * (x - px) + (y - py) * (y - py);
        return;
    }
    if (s.kind == MG_SEG_LINE) {
        double dx = s.p[2] - s.p[0], dy = s.p[3] - s.p[1];
        double L2 = dx * dx + dy * dy;
        t = L2 > 0 ? ((px - s.p[0]) * dx + (py - s.p[1]) * dy) / L2 : 0.0;
        t = std::min(1.0, std::max(0.0, t));
    } else {
        double th = std::atan2(py - s.p[1], px - s.p[0]);
        double t0 = s.p[3], sw = s.p[4] - s.p[3];
        // parameter of the angle th, unwrapped into the sweep if possible
        double u = (th - t0) / sw;
        double per = 2.0 * M_PI / std::fabs(sw);
        u -= per * std::floor(u / per);          // u in [0, per)
        if (u <= 1.0) {
            t = u;
        } else {
            // outside the arc: nearer end point
            double x0, y0, x1, y1;
            s.point(0.0, x0, y0);
            s.point(1.0, x1, y1);
            t = (std::hypot(px - x0, py - y0) <= std::hypot(px - x1, py - y1)) ? 0.0 : 1.0;
        }
    }
    double x, y;
    s.point(t, x, y);
    d2 = (x - px) * (x - px) + (y - py) * (y - py);
}

// in-place inverse by Gauss-Jordan with partial pivoting (row-major n x n)
bool invert_dense(int n, std::vector<double> &A) {
    std::vector<double> I((size_t)n * n, 0.0);
    for (int k = 0; k < n; ++k) I[(size_t)k * n + k] = 1.0;
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int r = k + 1; r < n; ++r)
            if (std::fabs(A[(size_t)r * n + k]) > std::fabs(A[(size_t)p * n + k])) p = r;
        if (A[(size_t)p * n + k] == 0.0) return false;
        if (p != k)
            for (int c = 0; c < n; ++c) {
                std::swap(A[(size_t)k * n + c], A[(size_t)p * n + c]);
                std::swap(I[(size_t)k * n + c], I[(size_t)p * n + c]);
            }
        double inv = 1.0 / A[(size_t)k * n + k];
        for (int c = 0; c < n; ++c) {
            A[(size_t)k * n + c] *= inv;
            I[(size_t)k * n + c] *= inv;
        }
#pragma omp parallel for schedule(static)
        for (int r = 0; r < n; ++r) {
            if (r == k) continue;
            double f = A[(size_t)r * n + k];
            if (f == 0.0) continue;
            double *ar = &A[(size_t)r * n], *ir = &I[(size_t)r * n];
            const double *ak = &A[(size_t)k * n], *ik = &I[(size_t)k * n];
            for (int c = 0; c < n; ++c) {
                ar[c] -= f * ak[c];
                ir[c] -= f * ik[c];
            }
        }
    }
    A.swap(I);
    return true;
}

}  // namespace

void build_plg_solver(const Level &L, int seg_max, PlgSolver &S) {
    const int nx = L.g.nx;
    const int m = (int)L.plg_cells.size();
    S = PlgSolver();
    S.m = m;
    if (m == 0) return;
    const auto &curves = L.curves->c;
    // Definition 5.1 ordering.  Cells whose closest point is a corner of
    // the curve (a segment end, as at the sharp tips of a star) share one
    // curve parameter; they are ordered by the angle of the cell centre
    // around the corner, swept from the incoming segment's side of Omega to
    // the outgoing one's, so that the chain stays banded around the corner.
    struct Key { int curve; double s, s2; int cell; };
    std::vector<Key> keys(m);
    for (int r = 0; r < m; ++r) {
        int cell = L.plg_cells[r];
        double px = L.g.x0 + (cell % nx + 0.5) * L.g.h, py = L.g.y0 + (cell / nx + 0.5) * L.g.h;
        double best = 1e300, best_t = 0.0;
        int best_seg = 0;
        Key k{0, 0.0, 0.0, cell};
        // PLG cells arise near the holes; the box is grid-aligned (ghost cells)
        for (size_t ci = curves.size() > 1 ? 1 : 0; ci < curves.size(); ++ci)
            for (size_t si = 0; si < curves[ci].size(); ++si) {
                double d2, t;
                closest_on_seg(curves[ci][si], px, py, d2, t);
                if (d2 < best) {
                    best = d2;
                    best_t = t;
                    best_seg = (int)si;
                    k.curve = (int)ci;
                    k.s = (si + t) / curves[ci].size();
                }
            }
        if (best_t <= 0.0 || best_t >= 1.0) {
            const auto &cv = curves[k.curve];
            const int nseg = (int)cv.size();
            const int sin_ = best_t >= 1.0 ? best_seg : (best_seg + nseg - 1) % nseg;   // incoming segment
            double ax, ay, dx, dy;
            cv[sin_].point(1.0, ax, ay);
            cv[sin_].deriv(1.0, dx, dy);
            const double nlx = -dy, nly = dx;                       // Omega's side of the incoming segment
            const double vx = px - ax, vy = py - ay;
            double cw = -std::atan2(nlx * vy - nly * vx, nlx * vx + nly * vy);
            if (cw < 0.0) cw += 2.0 * M_PI;
            k.s = (double)((best_t >= 1.0 ? best_seg + 1 : best_seg) % nseg) / nseg;
            k.s2 = cw;
        }
        keys[r] = k;
    }
    std::vector<int> order(m);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        if (keys[a].curve != keys[b].curve) return keys[a].curve < keys[b].curve;
        if (keys[a].s != keys[b].s) return keys[a].s < keys[b].s;
        if (keys[a].s2 != keys[b].s2) return keys[a].s2 < keys[b].s2;
        return keys[a].cell < keys[b].cell;
    });
    std::vector<int> pos(m);
    for (int k = 0; k < m; ++k) pos[order[k]] = k;
    // A22 couplings in the curve order: for each ordered position, the PLG
    // columns of its row
    std::vector<std::vector<std::pair<int, double>>> a22(m);
    for (int r = 0; r < m; ++r)
        for (int e = L.row_ptr[r]; e < L.row_ptr[r + 1]; ++e) {
            int pr = L.plg_row[L.col[e]];
            if (pr >= 0) a22[pos[r]].push_back({pos[pr], L.val[e]});
        }
    // chains per curve and bandwidth
    std::vector<int> chain_of(m);
    std::vector<std::pair<int, int>> chains;
    for (int k = 0; k < m;) {
        int c = keys[order[k]].curve, k1 = k;
        while (k1 < m && keys[order[k1]].curve == c) ++k1;
        for (int q = k; q < k1; ++q) chain_of[q] = (int)chains.size();
        chains.push_back({k, k1});
        k = k1;
    }
    std::vector<int> seg_of(m, -1);                 // -1 = separator
    int nseg = 0;
    for (auto &ch : chains) {
        int len = ch.second - ch.first;
        if (len <= seg_max) {
            for (int q = ch.first; q < ch.second; ++q) seg_of[q] = nseg;
            ++nseg;
            continue;
        }
        // reach[q]: the farthest in-chain coupling of position q (either
        // direction, wrap-around couplings excluded); a separator run at a
        // cut only needs to cover the couplings near that cut, so its length
        // is the largest reach within the global bandwidth w of the cut (a
        // few corner cells with long couplings, as at the tips of a star,
        // then lengthen only the runs next to them)
        std::vector<int> reach(len, 0);
        int w = 1;
        for (int q = ch.first; q < ch.second; ++q)
            for (auto &e : a22[q])
                if (chain_of[e.first] == chain_of[q]) {
                    int d = std::abs(e.first - q);
                    if (d < len / 2) {
                        w = std::max(w, d);
                        reach[q - ch.first] = std::max(reach[q - ch.first], d);
                        reach[e.first - ch.first] = std::max(reach[e.first - ch.first], d);
                    }
                }
        auto run_at = [&](int e) {                  // separator run length at position e
            int r = 1;
            for (int k = std::max(ch.first, e - w); k < std::min(ch.second, e + w); ++k)
                r = std::max(r, reach[k - ch.first]);
            return r;
        };
        int q = ch.first + run_at(ch.first);        // separator at the chain start
        while (q < ch.second) {
            int e = std::min(ch.second, q + seg_max - run_at(q + seg_max));
            e = std::max(e, std::min(ch.second, q + 1));
            if (ch.second - e < seg_max / 4) e = ch.second;   // no tiny tail segment
            for (int k = q; k < e; ++k) seg_of[k] = nseg;
            ++nseg;
            q = e + run_at(e);                      // next separator run
        }
    }
    // any coupling between different segments moves its column to S
    bool changed = true;
    while (changed) {
        changed = false;
        for (int q = 0; q < m; ++q) {
            if (seg_of[q] < 0) continue;
            for (auto &e : a22[q])
                if (seg_of[e.first] >= 0 && seg_of[e.first] != seg_of[q]) {
                    seg_of[e.first] = -1;
                    changed = true;
                }
        }
    }
    // final order: segments (curve order inside), then separators
    std::vector<std::vector<int>> segpos(nseg);
    std::vector<int> seppos;
    for (int q = 0; q < m; ++q) {
        if (seg_of[q] >= 0) segpos[seg_of[q]].push_back(q);
        else seppos.push_back(q);
    }
    S.seg_start.push_back(0);
    std::vector<int> newpos(m, -1);
    for (auto &sp : segpos) {
        if (sp.empty()) continue;
        for (int q : sp) {
            newpos[q] = (int)S.order.size();
            S.order.push_back(order[q]);
        }
        S.seg_start.push_back((int)S.order.size());
    }
    S.nseg = (int)S.seg_start.size() - 1;
    S.nsep = (int)seppos.size();
    S.sep_begin = (int)S.order.size();
    for (int q : seppos) {
        newpos[q] = (int)S.order.size();
        S.order.push_back(order[q]);
    }
    // dense blocks
    const int nb = S.nseg, ns = S.nsep, sb = S.sep_begin;
    std::vector<std::vector<std::pair<int, double>>> A(m);   // rows/cols in final order
    for (int q = 0; q < m; ++q)
        for (auto &e : a22[q]) A[newpos[q]].push_back({newpos[e.first], e.second});
    S.inv_off.assign(nb + 1, 0);
    S.f_off.assign(nb + 1, 0);
    S.fcols_ptr.assign(nb + 1, 0);
    for (int j = 0; j < nb; ++j) {
        long long Lj = S.seg_start[j + 1] - S.seg_start[j];
        S.inv_off[j + 1] = S.inv_off[j] + Lj * Lj;
    }
    S.inv.assign(S.inv_off[nb], 0.0);
    std::vector<std::vector<int>> fcols(nb);
    std::vector<double> Sp((size_t)ns * ns, 0.0);
    for (int r = sb; r < m; ++r)
        for (auto &e : A[r])
            if (e.first >= sb) Sp[(size_t)(r - sb) * ns + (e.first - sb)] += e.second;
    std::vector<std::vector<double>> Fj(nb);
    bool singular = false;
#pragma omp parallel for schedule(dynamic)
    for (int j = 0; j < nb; ++j) {
        int s0 = S.seg_start[j], Lj = S.seg_start[j + 1] - s0;
        std::vector<double> B((size_t)Lj * Lj, 0.0);
        std::vector<int> cols;
        for (int r = s0; r < s0 + Lj; ++r)
            for (auto &e : A[r]) {
                if (e.first >= s0 && e.first < s0 + Lj) B[(size_t)(r - s0) * Lj + (e.first - s0)] += e.second;
                else if (e.first >= sb) cols.push_back(e.first - sb);
            }
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        if (!invert_dense(Lj, B)) {
#pragma omp critical
            singular = true;
            continue;
        }
        // stored row-major
        double *dst = &S.inv[S.inv_off[j]];
        for (size_t e = 0; e < (size_t)Lj * Lj; ++e) dst[e] = B[e];
        // F = B^{-1} A_{j,S}
        int k = (int)cols.size();
        std::vector<double> AS((size_t)Lj * k, 0.0);
        for (int r = s0; r < s0 + Lj; ++r)
            for (auto &e : A[r])
                if (e.first >= sb) {
                    int kk = (int)(std::lower_bound(cols.begin(), cols.end(), e.first - sb) - cols.begin());
                    AS[(size_t)(r - s0) * k + kk] += e.second;
                }
        std::vector<double> F((size_t)Lj * k, 0.0);
        for (int r = 0; r < Lj; ++r)
            for (int c = 0; c < Lj; ++c) {
                double v = B[(size_t)r * Lj + c];
                if (v == 0.0) continue;
                for (int kk = 0; kk < k; ++kk) F[(size_t)r * k + kk] += v * AS[(size_t)c * k + kk];
            }
        Fj[j] = F;
        fcols[j] = cols;
    }
    if (singular) fail(MG_ERR_SINGULAR, "a PLG segment block is singular");
    for (int j = 0; j < nb; ++j) {
        int Lj = S.seg_start[j + 1] - S.seg_start[j], k = (int)fcols[j].size();
        S.f_off[j + 1] = S.f_off[j] + (long long)Lj * k;
        S.fcols_ptr[j + 1] = S.fcols_ptr[j] + k;
    }
    S.F.assign(S.f_off[nb], 0.0);
    S.fcols.clear();
    for (int j = 0; j < nb; ++j) {
        int Lj = S.seg_start[j + 1] - S.seg_start[j], k = (int)fcols[j].size();
        // row-major: F[r * k + kk]
        for (size_t e = 0; e < (size_t)Lj * k; ++e) S.F[S.f_off[j] + e] = Fj[j][e];
        for (int c : fcols[j]) S.fcols.push_back(c);
        // Schur complement: S' -= A_{S,j} F_j
        int s0 = S.seg_start[j];
        for (int r = sb; r < m; ++r)
            for (auto &e : A[r])
                if (e.first >= s0 && e.first < s0 + Lj) {
                    int lr = e.first - s0;
                    for (int kk = 0; kk < k; ++kk)
                        Sp[(size_t)(r - sb) * ns + fcols[j][kk]] -= e.second * Fj[j][(size_t)lr * k + kk];
                }
    }
    if (ns > 0) {
        if (!invert_dense(ns, Sp)) fail(MG_ERR_SINGULAR, "the PLG separator block is singular");
        S.sinv = Sp;                                // row-major
    }
    // separator rows: couplings to segment unknowns (positions < sb)
    S.sb_ptr.assign(ns + 1, 0);
    for (int r = sb; r < m; ++r) {
        for (auto &e : A[r])
            if (e.first < sb) {
                S.sb_col.push_back(e.first);
                S.sb_val.push_back(e.second);
            }
        S.sb_ptr[r - sb + 1] = (int)S.sb_col.size();
    }
}

}  // namespace mgc

namespace mgc {

void build_plg_plan(const Level &L, const PlgSolver &S, int nx, int slice, int bslice, int sep_group,
                    int sep_rows, PlgPlan &P) {
    P = PlgPlan();
    const int m = S.m;
    auto padded = [nx](int cell) { return (cell / nx + 2) * (nx + 4) + (cell % nx + 2); };
    // groups: the segments, then the separators in runs of sep_group rows
    P.grp_start.push_back(0);
    for (int j = 0; j < S.nseg; ++j) P.grp_start.push_back(S.seg_start[j + 1]);
    for (int s = S.sep_begin; s < m; s += sep_group) P.grp_start.push_back(std::min(m, s + sep_group));
    P.ngroup = (int)P.grp_start.size() - 1;
    // H of each group and the A21 rows in group-local numbering
    P.hptr.push_back(0);
    P.a21_loc.assign((size_t)m * ELL_W, 0);
    P.a21_val.assign((size_t)m * ELL_W, 0.0);
    for (int g = 0; g < P.ngroup; ++g) {
        std::vector<int> seen;                         // cells of H, first-appearance order
        for (int q = P.grp_start[g]; q < P.grp_start[g + 1]; ++q) {
            const int r = S.order[q];
            int k = 0;
            for (int e = L.row_ptr[r]; e < L.row_ptr[r + 1]; ++e) {
                const int c = L.col[e];
                if (L.kind[c] != 1) continue;
                int loc = (int)(std::find(seen.begin(), seen.end(), c) - seen.begin());
                if (loc == (int)seen.size()) seen.push_back(c);
                if (k == ELL_W) fail(MG_ERR_UNSUPPORTED, "a PLG row has more SFV couplings than the row width");
                P.a21_loc[(size_t)q * ELL_W + k] = loc;
                P.a21_val[(size_t)q * ELL_W + k] = L.val[e];
                ++k;
            }
        }
        for (int c : seen) P.hcell.push_back(padded(c));
        P.hptr.push_back((int)P.hcell.size());
        P.hmax = std::max(P.hmax, (int)seen.size());
        P.lmax = std::max(P.lmax, P.grp_start[g + 1] - P.grp_start[g]);
    }
    // padded segment inverses
    auto pad4 = [](int n) { return (n + 3) & ~3; };
    P.inv_off.assign(S.nseg + 1, 0);
    for (int j = 0; j < S.nseg; ++j) {
        const int Lj = S.seg_start[j + 1] - S.seg_start[j], Lp = pad4(Lj);
        P.inv_off[j + 1] = P.inv_off[j] + (long long)Lj * Lp;
    }
    P.INV.assign(P.inv_off[S.nseg], 0.0);
    for (int j = 0; j < S.nseg; ++j) {
        const int Lj = S.seg_start[j + 1] - S.seg_start[j], Lp = pad4(Lj);
        for (int r = 0; r < Lj; ++r)
            for (int c = 0; c < Lj; ++c)
                P.INV[P.inv_off[j] + (size_t)r * Lp + c] = S.inv[S.inv_off[j] + (size_t)r * Lj + c];
    }
    // launch A blocks (the A_SB ranges are filled in below)
    for (int g = 0; g < P.ngroup; ++g) {
        const int g0 = P.grp_start[g], g1 = P.grp_start[g + 1];
        const int step = g < S.nseg ? slice : g1 - g0;
        for (int r = g0; r < g1; r += step) {
            PlgBlkA b{};
            b.g = g; b.r0 = r; b.r1 = std::min(g1, r + step); b.gs = g0; b.n = g1 - g0;
            b.h0 = P.hptr[g]; b.nh = P.hptr[g + 1] - P.hptr[g];
            b.inv_off = g < S.nseg ? P.inv_off[g] : 0;
            P.blk1.push_back(b);
        }
    }
    if (S.nsep == 0) return;

    // A_SB entries owned by each segment, in ELL slots of the separator rows
    std::vector<int> seg_of(S.sep_begin);
    for (int j = 0, q = 0; q < S.sep_begin; ++q) {
        while (q >= S.seg_start[j + 1]) ++j;
        seg_of[q] = j;
    }
    std::vector<std::vector<std::array<int, 2>>> own(S.nseg);   // (slot, entry)
    for (int s = 0; s < S.nsep; ++s) {
        if (S.sb_ptr[s + 1] - S.sb_ptr[s] > ELL_W)
            fail(MG_ERR_UNSUPPORTED, "a separator row has more segment couplings than the row width");
        for (int e = S.sb_ptr[s]; e < S.sb_ptr[s + 1]; ++e)
            own[seg_of[S.sb_col[e]]].push_back({s * ELL_W + (e - S.sb_ptr[s]), e});
    }
    P.ce_ptr.push_back(0);
    for (int j = 0; j < S.nseg; ++j) {
        for (auto &se : own[j]) {
            P.ce_row.push_back(S.sb_col[se[1]]);
            P.ce_slot.push_back(se[0]);
            P.ce_val.push_back(S.sb_val[se[1]]);
        }
        P.ce_ptr.push_back((int)P.ce_row.size());
    }
    // S'^{-1}, F_j^T and the rows of S'^{-1} that segment j needs
    const int nsp = pad4(S.nsep);
    P.SINV.assign((size_t)S.nsep * nsp, 0.0);
    for (int r = 0; r < S.nsep; ++r)
        for (int c = 0; c < S.nsep; ++c) P.SINV[(size_t)r * nsp + c] = S.sinv[(size_t)r * S.nsep + c];
    P.ft_off.assign(S.nseg + 1, 0);
    P.sj_off.assign(S.nseg + 1, 0);
    P.FT.assign(S.F.size(), 0.0);
    for (int j = 0; j < S.nseg; ++j) {
        const int Lj = S.seg_start[j + 1] - S.seg_start[j], k = S.fcols_ptr[j + 1] - S.fcols_ptr[j];
        P.ft_off[j + 1] = P.ft_off[j] + (long long)Lj * k;
        P.sj_off[j + 1] = P.sj_off[j] + (long long)k * nsp;
        for (int r = 0; r < Lj; ++r)
            for (int kk = 0; kk < k; ++kk)
                P.FT[P.ft_off[j] + (size_t)kk * Lj + r] = S.F[S.f_off[j] + (size_t)r * k + kk];
        for (int kk = 0; kk < k; ++kk) {
            const int row = S.fcols[S.fcols_ptr[j] + kk];
            P.SJ.insert(P.SJ.end(), P.SINV.begin() + (size_t)row * nsp, P.SINV.begin() + (size_t)(row + 1) * nsp);
        }
        P.kmax = std::max(P.kmax, k);
    }
    for (auto &b : P.blk1)
        if (b.g < S.nseg) {
            b.ce0 = P.ce_ptr[b.g];
            b.ce1 = P.ce_ptr[b.g + 1];
        }
    // launch B blocks: the segments in slices of bslice rows, then separator
    // rows in runs (more blocks shorten the longest block's dense products,
    // which bound the launch, although each block forms all of r_S)
    for (int j = 0; j < S.nseg; ++j)
        for (int r = S.seg_start[j]; r < S.seg_start[j + 1]; r += bslice) {
            PlgBlkB b{};
            b.kind = 0; b.j = j; b.r0 = r; b.r1 = std::min(S.seg_start[j + 1], r + bslice);
            b.kj = S.fcols_ptr[j + 1] - S.fcols_ptr[j]; b.s0 = S.seg_start[j]; b.Lj = S.seg_start[j + 1] - S.seg_start[j];
            b.sj_off = P.sj_off[j]; b.ft_off = P.ft_off[j];
            P.blk2.push_back(b);
        }
    for (int s = 0; s < S.nsep; s += sep_rows) {
        PlgBlkB b{};
        b.kind = 1; b.r0 = s; b.r1 = std::min(S.nsep, s + sep_rows);
        P.blk2.push_back(b);
    }
}

namespace {

// x = A22^{-1} t (transpose = false) or x = A22^{-T} t, both in solve order:
// A22 = [B E; C D] with B the segment blocks, E = A_BS, C = A_SB (the
// separator rows' couplings), S' = D - C B^{-1} E, F = B^{-1} E.
//   A22 x = t:   y = B^{-1} t_B, x_S = S'^{-1} (t_S - C y), x_B = y - F x_S
//   A22^T z = w: z_S = S'^{-T} (w_S - F^T w_B), z_B = B^{-T} (w_B - C^T z_S)
std::vector<double> plg_apply_inverse(const PlgSolver &S, const std::vector<double> &t, bool transpose) {
    const int m = S.m, sb = S.sep_begin, ns = S.nsep;
    std::vector<double> x(m, 0.0), xs(ns, 0.0), rs(ns, 0.0);
    auto seg_mul = [&](int j, const double *in, double *out, bool tr) {
        const int s0 = S.seg_start[j], Lj = S.seg_start[j + 1] - s0;
        const double *B = &S.inv[S.inv_off[j]];
        for (int r = 0; r < Lj; ++r) out[r] = 0.0;
        for (int r = 0; r < Lj; ++r)
            for (int c = 0; c < Lj; ++c) {
                if (tr) out[c] += B[(size_t)r * Lj + c] * in[r];
                else out[r] += B[(size_t)r * Lj + c] * in[c];
            }
    };
    if (!transpose) {
        for (int j = 0; j < S.nseg; ++j) seg_mul(j, &t[S.seg_start[j]], &x[S.seg_start[j]], false);
        for (int s = 0; s < ns; ++s) {
            double v = t[sb + s];
            for (int e = S.sb_ptr[s]; e < S.sb_ptr[s + 1]; ++e) v -= S.sb_val[e] * x[S.sb_col[e]];
            rs[s] = v;
        }
        for (int s = 0; s < ns; ++s) {
            double v = 0.0;
            for (int c = 0; c < ns; ++c) v += S.sinv[(size_t)s * ns + c] * rs[c];
            xs[s] = v;
        }
        for (int j = 0; j < S.nseg; ++j) {
            const int s0 = S.seg_start[j], Lj = S.seg_start[j + 1] - s0, k = S.fcols_ptr[j + 1] - S.fcols_ptr[j];
            const double *F = &S.F[S.f_off[j]];
            for (int r = 0; r < Lj; ++r)
                for (int kk = 0; kk < k; ++kk) x[s0 + r] -= F[(size_t)r * k + kk] * xs[S.fcols[S.fcols_ptr[j] + kk]];
        }
        for (int s = 0; s < ns; ++s) x[sb + s] = xs[s];
        return x;
    }
    for (int s = 0; s < ns; ++s) rs[s] = t[sb + s];
    for (int j = 0; j < S.nseg; ++j) {
        const int s0 = S.seg_start[j], Lj = S.seg_start[j + 1] - s0, k = S.fcols_ptr[j + 1] - S.fcols_ptr[j];
        const double *F = &S.F[S.f_off[j]];
        for (int r = 0; r < Lj; ++r)
            for (int kk = 0; kk < k; ++kk) rs[S.fcols[S.fcols_ptr[j] + kk]] -= F[(size_t)r * k + kk] * t[s0 + r];
    }
    for (int c = 0; c < ns; ++c) {
        double v = 0.0;
        for (int s = 0; s < ns; ++s) v += S.sinv[(size_t)s * ns + c] * rs[s];
        xs[c] = v;
    }
    std::vector<double> g(t.begin(), t.begin() + sb);
    for (int s = 0; s < ns; ++s)
        for (int e = S.sb_ptr[s]; e < S.sb_ptr[s + 1]; ++e) g[S.sb_col[e]] -= S.sb_val[e] * xs[s];
    for (int j = 0; j < S.nseg; ++j) seg_mul(j, &g[S.seg_start[j]], &x[S.seg_start[j]], true);
    for (int s = 0; s < ns; ++s) x[sb + s] = xs[s];
    return x;
}

}  // namespace

double cond1_estimate(const Level &L, const PlgSolver &S) {
    const int m = S.m;
    if (m == 0) return 0.0;
    std::vector<int> pos(m);
    for (int q = 0; q < m; ++q) pos[S.order[q]] = q;
    std::vector<double> colsum(m, 0.0);
    for (int r = 0; r < m; ++r)
        for (int e = L.row_ptr[r]; e < L.row_ptr[r + 1]; ++e) {
            const int pr = L.plg_row[L.col[e]];
            if (pr >= 0) colsum[pos[pr]] += std::fabs(L.val[e]);
        }
    const double anorm = *std::max_element(colsum.begin(), colsum.end());
    auto norm1 = [](const std::vector<double> &v) {
        double s = 0.0;
        for (double x : v) s += std::fabs(x);
        return s;
    };
    std::vector<double> x(m, 1.0 / m);
    double est = 0.0;
    int last = -1;
    for (int it = 0; it < 5; ++it) {
        std::vector<double> y = plg_apply_inverse(S, x, false);
        const double e = norm1(y);
        if (it > 0 && e <= est) break;
        est = e;
        std::vector<double> xi(m);
        for (int q = 0; q < m; ++q) xi[q] = y[q] >= 0.0 ? 1.0 : -1.0;
        std::vector<double> z = plg_apply_inverse(S, xi, true);
        int jmax = 0;
        double zt = 0.0;
        for (int q = 0; q < m; ++q) {
            if (std::fabs(z[q]) > std::fabs(z[jmax])) jmax = q;
            zt += z[q] * x[q];
        }
        if (std::fabs(z[jmax]) <= zt || jmax == last) break;
        last = jmax;
        std::fill(x.begin(), x.end(), 0.0);
        x[jmax] = 1.0;
    }
    // Higham's extra test vector guards against the estimator's bad cases
    std::vector<double> alt(m);
    for (int q = 0; q < m; ++q) alt[q] = (q % 2 ? -1.0 : 1.0) * (1.0 + (m > 1 ? (double)q / (m - 1) : 0.0));
    est = std::max(est, 2.0 * norm1(plg_apply_inverse(S, alt, false)) / (3.0 * m));
    return anorm * est;
}

}  // namespace mgc
