// One level's linear system (Section 4): SFV/PLG classification
// (Definition 4.1), SFV rows with ghost cells eliminated (Section 4.1), poised
// lattices (Definitions 4.2-4.3; candidates ranked by a host fit of the
// actual row) and the inputs of the weighted minimum-norm fits
// (eqs. (4.10)-(4.18)); the fits used by the solver run on the GPU.

#include <algorithm>
#include <map>
#include <array>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "level.hpp"

namespace mgc {

// ---------------------------------------------------------------------------
// ghost weights (Section 4.1): (w_i, w_{i-1}, w_{i-2}, w_{i-3}, w_face) for
// the ghost 1 or 2 cells beyond the face.  The second Dirichlet face weight is
// 300/12: the value that reproduces all polynomials of degree <= 4.
void ghost_weights(int bc, int which, double w[5]) {
    static const double D[2][5] = {{-77.0 / 12, 43.0 / 12, -17.0 / 12, 3.0 / 12, 60.0 / 12},
                                   {-505.0 / 12, 335.0 / 12, -145.0 / 12, 27.0 / 12, 300.0 / 12}};
    static const double N[2][5] = {{5.0 / 10, 9.0 / 10, -5.0 / 10, 1.0 / 10, 12.0 / 10},
                                   {-15.0 / 2, 29.0 / 2, -15.0 / 2, 3.0 / 2, 12.0 / 2}};
    const double *src = (bc == MG_BC_DIRICHLET) ? D[which - 1] : N[which - 1];
    for (int k = 0; k < 5; ++k) w[k] = src[k];
}

// Ghost weights of a box face with the face datum g taken as given: g = u
// (Dirichlet), g = du/dn (Neumann: the face weight above times h), and
// g = alpha1 u + alpha2 du/dn (Robin).  Section 4.1 gives no Robin ghost; the
// reading: the degree-4 polynomial p in the normal coordinate x (cells of
// width 1, face at x = 0, interior cells i .. i-3 on [-1, 0] .. [-4, -3],
// outward normal +x) with those four cell averages and
// alpha1 p(0) + alpha2 p'(0) / h = g, averaged over the ghost cell
// [which - 1, which].
void face_ghost(int bc, double al1, double al2, double h, int which, double w[5]) {
    if (bc == MG_BC_PERIODIC) {            // no ghost formula: the kernels wrap instead
        for (int k = 0; k < 5; ++k) w[k] = 0.0;
        return;
    }
    if (bc != MG_BC_ROBIN) {
        ghost_weights(bc, which, w);
        if (bc == MG_BC_NEUMANN) w[4] *= h;
        return;
    }
    auto avg = [](double a, int k) { return (std::pow(a + 1.0, k + 1) - std::pow(a, k + 1)) / (k + 1); };
    // rows: conditions on the coefficients of p; w solves M^T w = e
    double A[5][6];
    for (int m = 0; m < 4; ++m)
        for (int k = 0; k < 5; ++k) A[k][m] = avg(-(m + 1.0), k);         // transposed
    for (int k = 0; k < 5; ++k) A[k][4] = k == 0 ? al1 : (k == 1 ? al2 / h : 0.0);
    for (int k = 0; k < 5; ++k) A[k][5] = avg(which - 1.0, k);
    for (int c = 0; c < 5; ++c) {                                          // Gauss-Jordan, partial pivoting
        int piv = c;
        for (int r = c + 1; r < 5; ++r)
            if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
        if (A[piv][c] == 0.0) fail(MG_ERR_INVALID_ARG, "Robin coefficients give no ghost formula");
        for (int k = 0; k < 6; ++k) std::swap(A[c][k], A[piv][k]);
        for (int r = 0; r < 5; ++r) {
            if (r == c) continue;
            const double f = A[r][c] / A[c][c];
            for (int k = c; k < 6; ++k) A[r][k] -= f * A[c][k];
        }
    }
    for (int k = 0; k < 5; ++k) w[k] = A[k][5] / A[k][k];
}

// Corner ghost (beyond the x-face by m cells and the y-face by k cells):
// the face-ghost formula of one face applied to the ghosts of the other,
// averaged over both orders; the face data beyond the corner are the cubic
// extrapolation of that face's data along the face.
void corner_weights(const CutGrid &cg, int xside, int yside, int m, int k, double h, double wu[4][4], double wgy[4],
                    double wgx[4]) {
    static const double E[2][4] = {{4, -6, 4, -1}, {10, -20, 15, -4}};
    double gx[5], gy[5];
    face_ghost(cg.box_bc[xside], cg.box_al[xside][0], cg.box_al[xside][1], h, m, gx);
    face_ghost(cg.box_bc[yside], cg.box_al[yside][0], cg.box_al[yside][1], h, k, gy);
    for (int p = 0; p < 4; ++p)
        for (int q = 0; q < 4; ++q) wu[p][q] = gx[p] * gy[q];
    for (int p = 0; p < 4; ++p) wgy[p] = 0.5 * gy[4] * (gx[p] + E[m - 1][p]);
    for (int q = 0; q < 4; ++q) wgx[q] = 0.5 * gx[4] * (gy[q] + E[k - 1][q]);
}

// SFV stencil of L = a d_xx + b d_xy + c d_yy, eq. (4.7) and the mixed term
void sfv_terms(double a, double b, double c, double h, std::vector<std::array<double, 3>> &terms) {
    static const double d1[5] = {1.0 / 12, -8.0 / 12, 0.0, 8.0 / 12, -1.0 / 12};
    static const double d2[5] = {-1.0 / 12, 16.0 / 12, -30.0 / 12, 16.0 / 12, -1.0 / 12};
    double w[5][5] = {};
    for (int m = 0; m < 5; ++m) {
        w[m][2] += a * d2[m];
        w[2][m] += c * d2[m];
    }
    if (b != 0.0)
        for (int m1 = 0; m1 < 5; ++m1)
            for (int m2 = 0; m2 < 5; ++m2) w[m1][m2] += b * d1[m1] * d1[m2];
    terms.clear();
    for (int m1 = 0; m1 < 5; ++m1)
        for (int m2 = 0; m2 < 5; ++m2)
            if (w[m1][m2] != 0.0) terms.push_back({(double)(m1 - 2), (double)(m2 - 2), w[m1][m2] / (h * h)});
}

int Level::face_index(int side, int k) const {
    switch (side) {
        case 0: return k;
        case 2: return g.nx + k;
        case 3: return 2 * g.nx + k;
        default: return 2 * g.nx + g.ny + k;
    }
}

// Row of an SFV cell with ghosts eliminated: coefficients on interior cells
// (cells[]) and on boundary data (gidx[]).
void Level::sfv_row(int i, int j, std::vector<std::pair<int, double>> &cells,
                    std::vector<std::pair<int, double>> &gdat) const {
    const int nx = g.nx, ny = g.ny;
    const double h = g.h;
    std::vector<std::array<double, 3>> terms;
    sfv_terms(a, b, c, h, terms);
    cells.clear();
    gdat.clear();
    // periodic box sides: positions beyond them are the cells one period
    // away; what is still outside takes the other sides' ghost formulas
    const bool per_x = cg.box_bc[1] == MG_BC_PERIODIC, per_y = cg.box_bc[0] == MG_BC_PERIODIC;
    for (auto &t : terms) {
        int qi = i + (int)t[0], qj = j + (int)t[1];
        if (per_x) qi = (qi % nx + nx) % nx;
        if (per_y) qj = (qj % ny + ny) % ny;
        double w = t[2];
        bool outx = qi < 0 || qi >= nx, outy = qj < 0 || qj >= ny;
        if (!outx && !outy) {
            cells.push_back({qj * nx + qi, w});
        } else if (outx && outy) {
            int xside = qi < 0 ? 3 : 1, yside = qj < 0 ? 0 : 2;
            int m = qi < 0 ? -qi : qi - nx + 1, k = qj < 0 ? -qj : qj - ny + 1;
            double wu[4][4], wgy[4], wgx[4];
            corner_weights(cg, xside, yside, m, k, h, wu, wgy, wgx);
            for (int p = 0; p < 4; ++p) {
                int col = xside == 3 ? p : nx - 1 - p;
                for (int q = 0; q < 4; ++q) {
                    int row = yside == 0 ? q : ny - 1 - q;
                    cells.push_back({row * nx + col, w * wu[p][q]});
                }
                gdat.push_back({face_index(yside, col), w * wgy[p]});
                int row = yside == 0 ? p : ny - 1 - p;
                gdat.push_back({face_index(xside, row), w * wgx[p]});
            }
        } else {
            int side, depth, along;
            if (qj < 0) { side = 0; depth = -qj; along = qi; }
            else if (qj >= ny) { side = 2; depth = qj - ny + 1; along = qi; }
            else if (qi < 0) { side = 3; depth = -qi; along = qj; }
            else { side = 1; depth = qi - nx + 1; along = qj; }
            double gw[5];
            face_ghost(cg.box_bc[side], cg.box_al[side][0], cg.box_al[side][1], h, depth, gw);
            for (int k = 0; k < 4; ++k) {
                int ci, cj;
                if (side == 0) { ci = along; cj = k; }
                else if (side == 2) { ci = along; cj = ny - 1 - k; }
                else if (side == 3) { ci = k; cj = along; }
                else { ci = nx - 1 - k; cj = along; }
                cells.push_back({cj * nx + ci, w * gw[k]});
            }
            gdat.push_back({face_index(side, along), w * gw[4]});
        }
    }
}

// ---------------------------------------------------------------------------
// Definition 4.1
void Level::classify() {
    const int nx = g.nx, ny = g.ny;
    if (nx < 4 || ny < 4) fail(MG_ERR_GEOMETRY, "grid too small for ghost cells");
    const auto &R = cg.regular;
    for (int j = 0; j < ny; ++j)
        for (int k = 0; k < 4; ++k)
            if (!R[(size_t)j * nx + k] || !R[(size_t)j * nx + nx - 1 - k])
                fail(MG_ERR_GEOMETRY, "a box face is not extendable");
    for (int i = 0; i < nx; ++i)
        for (int k = 0; k < 4; ++k)
            if (!R[(size_t)k * nx + i] || !R[(size_t)(ny - 1 - k) * nx + i])
                fail(MG_ERR_GEOMETRY, "a box face is not extendable");
    // every position outside the box within 2 cells is a (face or corner) ghost
    auto ok = [&](int i, int j) {
        if (i >= 0 && i < nx && j >= 0 && j < ny) return (bool)R[(size_t)j * nx + i];
        return i >= -2 && i < nx + 2 && j >= -2 && j < ny + 2;
    };
    kind.assign((size_t)nx * ny, 0);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t cell = (size_t)j * nx + i;
            if (!cg.active[cell]) continue;
            bool sfv = true;
            if (b == 0.0) {
                for (int m = -2; m <= 2 && sfv; ++m) sfv = ok(i + m, j) && ok(i, j + m);
            } else {
                for (int m1 = -2; m1 <= 2 && sfv; ++m1)
                    for (int m2 = -2; m2 <= 2 && sfv; ++m2) sfv = ok(i + m1, j + m2);
            }
            kind[cell] = sfv ? 1 : 2;
        }
    plg_cells.clear();
    plg_row.assign((size_t)nx * ny, -1);
    for (int cell = 0; cell < nx * ny; ++cell)
        if (kind[cell] == 2) {
            plg_row[cell] = (int)plg_cells.size();
            plg_cells.push_back(cell);
        }
    n_active = 0;
    for (auto v : cg.active) n_active += v ? 1 : 0;
    n_face = 2 * nx + 2 * ny;
    g_of_cell.assign((size_t)nx * ny, -1);
    n_irr = 0;
    for (int cell = 0; cell < nx * ny; ++cell)
        if (cg.active[cell] && !cg.regular[cell]) g_of_cell[cell] = n_face + n_irr++;
}

// ---------------------------------------------------------------------------
// lattice selection
namespace {

constexpr uint64_t PRIME = (1ULL << 61) - 1;

uint64_t mulmod(uint64_t a, uint64_t b) { return (uint64_t)((unsigned __int128)a * b % PRIME); }
uint64_t powmod(uint64_t a, uint64_t e) {
    uint64_t r = 1;
    while (e) {
        if (e & 1) r = mulmod(r, a);
        a = mulmod(a, a);
        e >>= 1;
    }
    return r;
}
uint64_t tomod(long long v) {
    long long r = v % (long long)PRIME;
    return r < 0 ? (uint64_t)(r + (long long)PRIME) : (uint64_t)r;
}

// Incremental echelon form of point-sample rows [d^alpha] modulo the prime
// 2^61 - 1.  Rows independent modulo a prime are independent over the
// rationals; the converse fails only if the prime divides a nonzero minor of
// integers below 4^60, which does not happen for these small lattices.
struct Echelon {
    std::vector<std::pair<int, std::array<uint64_t, NB>>> rows;
    bool try_add(int dx, int dy) {
        std::array<uint64_t, NB> v;
        for (int k = 0; k < NB; ++k) {
            long long t = 1;
            for (int a = 0; a < MONO_P[k]; ++a) t *= dx;
            for (int b = 0; b < MONO_Q[k]; ++b) t *= dy;
            v[k] = tomod(t);
        }
        for (auto &pr : rows) {
            int pv = pr.first;
            if (v[pv] == 0) continue;
            uint64_t f = mulmod(v[pv], powmod(pr.second[pv], PRIME - 2));
            for (int k = 0; k < NB; ++k) v[k] = (v[k] + PRIME - mulmod(f, pr.second[k])) % PRIME;
        }
        for (int k = 0; k < NB; ++k)
            if (v[k]) {
                rows.push_back({k, v});
                return true;
            }
        return false;
    }
};

double angle_of(int x, int y) {
    double t = std::atan2((double)y, (double)x);
    if (t < 0) t += 2.0 * M_PI;
    return t;
}

// Weighted minimum-norm fit of eqs. (4.16)-(4.18) on the host, used to rank
// candidate lattices: beta = W^{1/2} gamma with gamma the minimum-2-norm
// solution of (M W^{1/2}) gamma = phibar, W = diag(1 / w_k).  M is column-major
// (NB rows, ncol columns).  Householder QR of (M W^{1/2})^T = Q R, then
// gamma = Q R^{-T} phibar.  Returns false for a rank-deficient M.
bool host_fit(int ncol, const double *M, const double *phi, const double *w, double *beta) {
    double A[(NB + 1) * NB];                      // A[k * NB + q] = M[q, k] / sqrt(w_k)
    double v[NB][NB + 1], tau[NB];
    for (int k = 0; k < ncol; ++k)
        for (int q = 0; q < NB; ++q) A[k * NB + q] = M[(size_t)k * NB + q] / std::sqrt(w[k]);
    for (int q = 0; q < NB; ++q) {
        double nrm = 0.0;
        for (int k = q; k < ncol; ++k) nrm += A[k * NB + q] * A[k * NB + q];
        nrm = std::sqrt(nrm);
        if (nrm == 0.0) return false;
        double alpha = A[q * NB + q] > 0 ? -nrm : nrm;
        for (int k = 0; k < ncol; ++k) v[q][k] = k < q ? 0.0 : A[k * NB + q];
        v[q][q] -= alpha;
        double vv = 0.0;
        for (int k = q; k < ncol; ++k) vv += v[q][k] * v[q][k];
        tau[q] = vv > 0.0 ? 2.0 / vv : 0.0;
        for (int c = q; c < NB; ++c) {
            double d = 0.0;
            for (int k = q; k < ncol; ++k) d += v[q][k] * A[k * NB + c];
            d *= tau[q];
            for (int k = q; k < ncol; ++k) A[k * NB + c] -= d * v[q][k];
        }
    }
    // R^T z = phibar (R = upper triangle of A's first NB rows)
    double g[NB + 1] = {};
    for (int q = 0; q < NB; ++q) {
        double s = phi[q];
        for (int k = 0; k < q; ++k) s -= A[k * NB + q] * g[k];
        if (A[q * NB + q] == 0.0) return false;
        g[q] = s / A[q * NB + q];
    }
    // gamma = H_0 ... H_{NB-1} [z; 0]
    for (int q = NB - 1; q >= 0; --q) {
        double d = 0.0;
        for (int k = q; k < ncol; ++k) d += v[q][k] * g[k];
        d *= tau[q];
        for (int k = q; k < ncol; ++k) g[k] -= d * v[q][k];
    }
    for (int k = 0; k < ncol; ++k) beta[k] = g[k] / std::sqrt(w[k]);
    return true;
}

// Ranking key of a fitted row whose lattice starts at the cell itself:
// sum_{k>0} |beta_k| / (-beta_0) when the cell's own coefficient is negative
// (the sign of the operator's diagonal), else +inf.
double row_dominance(const double *beta) {
    if (!(beta[0] < 0.0)) return INFINITY;
    double s = 0.0;
    for (int k = 1; k < NB; ++k) s += std::fabs(beta[k]);
    return s / -beta[0];
}

}  // namespace

// Candidate lattices S_PLG(i) (Definitions 4.2-4.3): K = active cells of the
// 7x7 box centred at i (9x9 if no poised subset exists).  For each of the 8
// grid symmetries g, take nodes nearest-first by (|d|^2, angle of g(d) in
// [0, 2pi)) when they raise the exact rank of the point-sample matrix
// [d^alpha], |alpha| <= 4, until 15.  Distinct lattices in symmetry order;
// each starts with d = (0, 0).
// the 9x9 activity pattern around (i, j): the candidates depend on nothing else
__uint128_t Level::lattice_key(int i, int j) const {
    const int nx = g.nx, ny = g.ny;
    __uint128_t key = 0;
    for (int dy = -4; dy <= 4; ++dy)
        for (int dx = -4; dx <= 4; ++dx) {
            int qi = i + dx, qj = j + dy;
            bool act = qi >= 0 && qi < nx && qj >= 0 && qj < ny && cg.active[(size_t)qj * nx + qi];
            key = (key << 1) | (act ? 1 : 0);
        }
    return key;
}

std::vector<std::vector<std::array<int, 2>>> Level::lattice_candidates(int i, int j) const {
    const int nx = g.nx, ny = g.ny;
    static const int SYM[8][4] = {{1, 0, 0, 1}, {0, -1, 1, 0}, {-1, 0, 0, -1}, {0, 1, -1, 0},
                                  {1, 0, 0, -1}, {0, 1, 1, 0}, {-1, 0, 0, 1}, {0, -1, -1, 0}};
    std::vector<std::vector<std::array<int, 2>>> out;
    for (int half : {3, 4}) {
        std::vector<std::array<int, 2>> box;
        for (int dy = -half; dy <= half; ++dy)
            for (int dx = -half; dx <= half; ++dx) {
                int qi = i + dx, qj = j + dy;
                if (qi >= 0 && qi < nx && qj >= 0 && qj < ny && cg.active[(size_t)qj * nx + qi]) box.push_back({dx, dy});
            }
        if ((int)box.size() < NB) continue;
        for (auto &s : SYM) {
            std::vector<std::pair<std::pair<int, double>, std::array<int, 2>>> ord;
            for (auto &d : box)
                ord.push_back({{d[0] * d[0] + d[1] * d[1], angle_of(s[0] * d[0] + s[1] * d[1], s[2] * d[0] + s[3] * d[1])}, d});
            std::sort(ord.begin(), ord.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
            Echelon ech;
            std::vector<std::array<int, 2>> lat;
            for (auto &o : ord) {
                if (ech.try_add(o.second[0], o.second[1])) lat.push_back(o.second);
                if ((int)lat.size() == NB) break;
            }
            if ((int)lat.size() < NB) continue;
            if (std::find(out.begin(), out.end(), lat) == out.end()) out.push_back(lat);
        }
        if (!out.empty()) break;
    }
    if (out.empty()) fail(MG_ERR_GEOMETRY, "no poised lattice for a PLG cell");
    return out;
}

// ---------------------------------------------------------------------------
// fit inputs: M (15 x ncol, column-major per cell), phibar, weights.  The
// lattice of each PLG cell is the candidate whose fitted row (host fit of the
// actual cell, its neighbours and B_i) has the smallest row_dominance; a key
// within a relative 1e-9 of the best so far keeps the earlier candidate, and
// with no negative own coefficient among them the first candidate is kept.
void Level::fit_inputs(std::vector<double> &Mall, std::vector<double> &phi, std::vector<double> &wall,
                       std::vector<int> &ncol) {
    const int nx = g.nx;
    const double h = g.h;
    const int m = (int)plg_cells.size();
    Mall.assign((size_t)m * NB * (NB + 1), 0.0);
    phi.assign((size_t)m * NB, 0.0);
    wall.assign((size_t)m * (NB + 1), 0.0);
    ncol.assign(m, NB);
    lattices.resize(m);
    // candidates: one search per distinct activity pattern, in parallel
    std::vector<__uint128_t> keys(m);
#pragma omp parallel for schedule(static)
    for (int r = 0; r < m; ++r) keys[r] = lattice_key(plg_cells[r] % nx, plg_cells[r] / nx);
    std::map<__uint128_t, int> first;                 // pattern -> first row with it
    std::vector<int> rep;
    for (int r = 0; r < m; ++r)
        if (first.emplace(keys[r], r).second) rep.push_back(r);
    std::vector<std::vector<std::vector<std::array<int, 2>>>> found(rep.size());
    int failed = 0;
#pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < (int)rep.size(); ++k) {
        try {
            found[k] = lattice_candidates(plg_cells[rep[k]] % nx, plg_cells[rep[k]] / nx);
        } catch (const status_error &) {
#pragma omp atomic write
            failed = 1;
        }
    }
    if (failed) fail(MG_ERR_GEOMETRY, "no poised lattice for a PLG cell");
    std::map<__uint128_t, int> slot;
    for (int k = 0; k < (int)rep.size(); ++k) slot[keys[rep[k]]] = k;
    std::vector<int> cand_of(m);
    for (int r = 0; r < m; ++r) cand_of[r] = slot[keys[r]];
    std::vector<double> gx, gw;
    gauss_legendre(16, gx, gw);
#pragma omp parallel for schedule(dynamic, 16)
    for (int r = 0; r < m; ++r) {
        int cell = plg_cells[r];
        int i = cell % nx, j = cell / nx;
        double *M = &Mall[(size_t)r * NB * (NB + 1)];
        double *w = &wall[(size_t)r * (NB + 1)];
        double mom[NB];
        cell_moments(cg, i, j, mom);
        for (int q = 0; q < NB; ++q) {
            int p = MONO_P[q], qq = MONO_Q[q];
            double s = 0.0;
            if (p >= 2) s += a * p * (p - 1) * mom[mono_index(p - 2, qq)];
            if (p >= 1 && qq >= 1) s += b * p * qq * mom[mono_index(p - 1, qq - 1)];
            if (qq >= 2) s += c * qq * (qq - 1) * mom[mono_index(p, qq - 2)];
            phi[(size_t)r * NB + q] = s / mom[0] / (h * h);
        }
        if (!cg.regular[cell]) {
            // boundary column <<N phi_alpha>>_{B_i}
            double xc = g.x0 + (i + 0.5) * h, yc = g.y0 + (j + 0.5) * h;
            double tot[NB] = {}, len = 0.0;
            const CellData &d = cg.irr[cg.irr_slot[cell]];
            for (auto &bp : d.bp) {
                const Seg &s = curves->c[bp.curve][bp.seg];
                for (int n = 0; n < 16; ++n) {
                    double t = 0.5 * (bp.tb - bp.ta) * gx[n] + 0.5 * (bp.ta + bp.tb);
                    double x, y, dx, dy;
                    s.point(t, x, y);
                    s.deriv(t, dx, dy);
                    double sp = std::hypot(dx, dy);
                    double ds = 0.5 * (bp.tb - bp.ta) * gw[n] * sp;
                    double nxv = dy / sp, nyv = -dx / sp;
                    double X = (x - xc) / h, Y = (y - yc) / h;
                    for (int q = 0; q < NB; ++q) {
                        int p = MONO_P[q], qq = MONO_Q[q];
                        double ph = std::pow(X, p) * std::pow(Y, qq);
                        double gxv = p >= 1 ? p * std::pow(X, p - 1) * std::pow(Y, qq) / h : 0.0;
                        double gyv = qq >= 1 ? qq * std::pow(X, p) * std::pow(Y, qq - 1) / h : 0.0;
                        double dn = gxv * nxv + gyv * nyv;
                        double val = s.bc == MG_BC_DIRICHLET ? ph : (s.bc == MG_BC_NEUMANN ? dn : s.al1 * ph + s.al2 * dn);
                        tot[q] += ds * val;
                    }
                    len += ds;
                }
            }
            for (int q = 0; q < NB; ++q) M[(size_t)NB * NB + q] = tot[q] / len;
            w[NB] = w_min;
            ncol[r] = NB + 1;
        }
        // rank the candidates by their fitted rows
        auto load = [&](const std::vector<std::array<int, 2>> &lat) {
            for (int k = 0; k < NB; ++k) {
                int qi = i + lat[k][0], qj = j + lat[k][1];
                double mk[NB], sh[NB];
                cell_moments(cg, qi, qj, mk);
                shift_moments(mk, lat[k][0], lat[k][1], sh);
                for (int q = 0; q < NB; ++q) M[(size_t)k * NB + q] = sh[q] / mk[0];
                w[k] = std::max(std::hypot((double)lat[k][0], (double)lat[k][1]), w_min);
            }
        };
        const auto &cands = found[cand_of[r]];
        int best = 0;
        double bestv = INFINITY;
        for (int cidx = 0; cidx < (int)cands.size() && cands.size() > 1; ++cidx) {
            load(cands[cidx]);
            double beta[NB + 1];
            if (!host_fit(ncol[r], M, &phi[(size_t)r * NB], w, beta)) continue;
            double v = row_dominance(beta);
            if (v < bestv * (1.0 - 1e-9)) {
                best = cidx;
                bestv = v;
            }
        }
        lattices[r] = cands[best];
        load(cands[best]);
    }
}

}  // namespace mgc
