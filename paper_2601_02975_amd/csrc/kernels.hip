// HIP kernels of the cut-cell V-cycle for CDNA4 (gfx950).
//
// Cell arrays are row-major with a halo of 2: cell (i, j) at
// (j + 2) * pitch + (i + 2), pitch = nx + 4.  The halo is never read as data:
// ghost values are synthesised from interior cells (Section 4.1).
//
// One block smoothing sweep (Definition 5.6) is two steps:
//   A: omega-Jacobi on the SFV cells (eq. (5.5)) in 64 x 32 (64 x 8 on small
//      grids) tiles, and, per group of PLG rows, t = b2 - A21 u1 (eq. (5.6))
//      from Jacobi-updated values of the SFV cells those rows couple to,
//      followed by the segment solves y = B^{-1} t.  One launch, in which
//      the PLG groups recompute those values from the old iterate (so that
//      the step needs no grid-wide ordering), or, from 2048^2 cells, a tile
//      kernel and then the PLG groups, which read them from its output;
//   B: the separator Schur-complement solve and the segment corrections
//      (only on levels with separators; two launches from 768 separators).
// Tiles and PLG blocks are handed to the 8 XCDs in runs of consecutive
// indices, so that neighbours share cache lines in one L2.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>

#include "kernels.hpp"
#include "kernels_launch.hpp"

namespace mgc {

__device__ __forceinline__ size_t pidx(const LevelArgs &L, int i, int j) {
    return (size_t)(j + 2) * L.pitch + (size_t)(i + 2);
}

// ghost weights of the level (a device array: indexing it at run time keeps
// the argument struct out of scratch memory)
struct GhostW {
    const LevelArgs &L;
    __device__ double operator()(int side, int depth, int k) const { return L.gw[(side * 2 + depth - 1) * 4 + k]; }
};

// ghost weights staged in LDS: w[side][depth - 1][k]
struct GhostWLds {
    const double *w;
    __device__ double operator()(int side, int depth, int k) const { return w[(side * 2 + depth - 1) * 4 + k]; }
};

// Ghost value at (qi, qj) outside the box (homogeneous part; face data live
// in the right-hand side), from in-box values at(i, j) and ghost weights
// W(side, depth, k).  Corner positions apply the x and y face formulas in
// turn.  Across a periodic side the position is first moved by one period.
template <typename T, typename At, typename Wt>
__device__ T ghost_at(const At &at, const Wt &W, const LevelArgs &L, int qi, int qj) {
    if (L.periodic & 1) qi = qi < 0 ? qi + L.nx : qi >= L.nx ? qi - L.nx : qi;
    if (L.periodic & 2) qj = qj < 0 ? qj + L.ny : qj >= L.ny ? qj - L.ny : qj;
    const bool ox = qi < 0 || qi >= L.nx, oy = qj < 0 || qj >= L.ny;
    if (!ox && !oy) return at(qi, qj);
    if (ox && oy) {
        const int xside = qi < 0 ? 3 : 1, yside = qj < 0 ? 0 : 2;
        const int m = qi < 0 ? -qi : qi - L.nx + 1, k = qj < 0 ? -qj : qj - L.ny + 1;
        double s = 0.0;
        for (int p = 0; p < 4; ++p) {
            const int col = xside == 3 ? p : L.nx - 1 - p;
            double t = 0.0;
            for (int q = 0; q < 4; ++q) t += W(yside, k, q) * (double)at(col, yside == 0 ? q : L.ny - 1 - q);
            s += W(xside, m, p) * t;
        }
        return (T)s;
    }
    int side, depth;
    if (qj < 0) { side = 0; depth = -qj; }
    else if (qj >= L.ny) { side = 2; depth = qj - L.ny + 1; }
    else if (qi < 0) { side = 3; depth = -qi; }
    else { side = 1; depth = qi - L.nx + 1; }
    double s = 0.0;
    for (int k = 0; k < 4; ++k) {
        double v;
        if (side == 0) v = (double)at(qi, k);
        else if (side == 2) v = (double)at(qi, L.ny - 1 - k);
        else if (side == 3) v = (double)at(k, qj);
        else v = (double)at(L.nx - 1 - k, qj);
        s += W(side, depth, k) * v;
    }
    return (T)s;
}

// value at (i, j), in the box or a ghost, read from global memory
template <typename T>
__device__ __forceinline__ T fetch(const T *__restrict__ u, const LevelArgs &L, int i, int j) {
    auto at = [&](int a, int c) { return u[pidx(L, a, c)]; };
    if (i >= 0 && i < L.nx && j >= 0 && j < L.ny) return at(i, j);
    return ghost_at<T>(at, GhostW{L}, L, i, j);
}

// (A u) at an SFV cell from a 2D accessor (eq. (4.7) and the mixed term)
template <typename T, bool MIXED, typename F>
__device__ __forceinline__ T apply_sfv(const LevelArgs &L, F at) {
    const T c0 = at(0, 0);
    T dxx = (-(at(-2, 0) + at(2, 0)) + (T)16 * (at(-1, 0) + at(1, 0)) - (T)30 * c0) * (T)(1.0 / 12.0);
    T dyy = (-(at(0, -2) + at(0, 2)) + (T)16 * (at(0, -1) + at(0, 1)) - (T)30 * c0) * (T)(1.0 / 12.0);
    T s = (T)L.cxx * dxx + (T)L.cyy * dyy;
    if (MIXED) {
        T dx[5];
#pragma unroll
        for (int m2 = -2; m2 <= 2; ++m2) {
            if (m2 == 0) { dx[2] = 0; continue; }
            dx[m2 + 2] = ((at(-2, m2) - at(2, m2)) + (T)8 * (at(1, m2) - at(-1, m2))) * (T)(1.0 / 12.0);
        }
        T dxy = ((dx[0] - dx[4]) + (T)8 * (dx[3] - dx[1])) * (T)(1.0 / 12.0);
        s += (T)L.cxy * dxy;
    }
    return s;
}

// (A u) at the SFV cell (i, j) from global memory: direct loads when its
// 5 x 5 box lies in the grid (all loads issue together), else through fetch
template <typename T, bool MIXED>
__device__ __forceinline__ T sfv_global(const LevelArgs &L, const T *__restrict__ u, int i, int j) {
    if (i >= 2 && i < L.nx - 2 && j >= 2 && j < L.ny - 2) {
        const T *p = u + pidx(L, i, j);
        const int pt = L.pitch;
        return apply_sfv<T, MIXED>(L, [&](int dx, int dy) { return p[dy * pt + dx]; });
    }
    return apply_sfv<T, MIXED>(L, [&](int dx, int dy) { return fetch(u, L, i + dx, j + dy); });
}

constexpr int TX = 64, TY = 32, HX = TX + 4, HY = TY + 4, NT = 256;
static_assert(PLG_SLICE <= NT && PLG_B_ROWS <= NT, "launch B holds one segment row per thread");

// Loads the (TY+4) x (TX+4) tile with halo into LDS from in-box values
// at(i, j); halo positions outside the box get ghost values.  A block at the
// box edge first loads the interior cells and the ghost weights, then
// computes the ghosts of its part of the 2-cell band around the box from
// LDS when the 4 cells inward from each edge it touches lie in the tile
// (always so when at least 2 cells of the box remain in the last tile), else
// from the accessor.  gws: 32 doubles of LDS for the weights.
template <typename T, typename At, int TYv = TY>
__device__ __forceinline__ void load_tile(T (*s)[HX], double *gws, const At &at, const LevelArgs &L, int i0, int j0) {
    constexpr int HYv = TYv + 4;
    const bool edge = i0 < 2 || j0 < 2 || i0 + TX + 2 > L.nx || j0 + TYv + 2 > L.ny;
    if (edge && threadIdx.x < 32) gws[threadIdx.x] = L.gw[threadIdx.x];
    // all global loads of a thread are issued before any LDS store
    constexpr int NL = (HX * HYv + NT - 1) / NT;
    T v[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int t = threadIdx.x + k * NT;
        const int ly = t / HX, lx = t - ly * HX;
        const int qi = i0 - 2 + lx, qj = j0 - 2 + ly;
        v[k] = (t < HX * HYv && qi >= 0 && qi < L.nx && qj >= 0 && qj < L.ny) ? at(qi, qj) : (T)0;
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int t = threadIdx.x + k * NT;
        if (t < HX * HYv) s[t / HX][t % HX] = v[k];
    }
    if (!edge) return;
    // the tile holds cells [i0 - 2, i0 + TX + 2) x [j0 - 2, j0 + TY + 2)
    // (periodic sides wrap to cells that may lie outside the tile)
    const bool lds_ok = !L.periodic && (i0 + TX + 2 <= L.nx || L.nx - 4 >= i0 - 2) &&
                        (j0 + TYv + 2 <= L.ny || L.ny - 4 >= j0 - 2);
    auto lat = [&](int i, int j) { return s[j - j0 + 2][i - i0 + 2]; };
    const GhostWLds W{gws};
    __syncthreads();
    // the ghost band: columns -2, -1, nx, nx+1 over rows -2 .. ny+1, then
    // rows -2, -1, ny, ny+1 over columns 0 .. nx-1; positions outside the
    // tile are skipped
    constexpr int NV = 2 * (HYv), NH = 2 * (HX);
    for (int t = threadIdx.x; t < 2 * NV + 2 * NH; t += NT) {
        int qi, qj;
        bool ok;
        if (t < 2 * NV) {
            const int band = t / NV, r = t - band * NV;          // band 0 left, 1 right
            const int c = r / HYv;
            qi = band == 0 ? -2 + c : L.nx + c;
            qj = j0 - 2 + (r - c * HYv);
            ok = qj >= -2 && qj < L.ny + 2;
        } else {
            const int t2 = t - 2 * NV;
            const int band = t2 / NH, r = t2 - band * NH;        // band 0 bottom, 1 top
            const int c = r / HX;
            qj = band == 0 ? -2 + c : L.ny + c;
            qi = i0 - 2 + (r - c * HX);
            ok = qi >= 0 && qi < L.nx;
        }
        const int lx = qi - i0 + 2, ly = qj - j0 + 2;
        if (ok && lx >= 0 && lx < HX && ly >= 0 && ly < HYv)
            s[ly][lx] = lds_ok ? ghost_at<T>(lat, W, L, qi, qj) : ghost_at<T>(at, W, L, qi, qj);
    }
}

// 16-byte vector of T
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    using V = float4;
    static constexpr int N = 4;
    __device__ static float at(const V &v, int k) { return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w; }
};
template <>
struct Vec16<double> {
    using V = double2;
    static constexpr int N = 2;
    __device__ static double at(const V &v, int k) { return k == 0 ? v.x : v.y; }
};

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Rows [0, nr) (nr <= 8) of a row-major block A with row stride lda (a
// multiple of 4) times x (LDS, zero beyond the last column up to lda), one
// wavefront: each lane loads 16 bytes of every row per step, U steps per
// pass so that a row of up to 64 * U * (16 / sizeof(T)) columns is read by
// loads issued together.  Lane 0 receives the 8 results.
template <typename T, int U>
__device__ __forceinline__ void wave_rows8(const T *__restrict__ A, int lda, int nr, const T *x, int lane, T out[8]) {
    using VT = Vec16<T>;
    using V = typename VT::V;
    constexpr int VN = VT::N;
    T acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0;
    for (int base = lane * VN; base < lda; base += 64 * VN * U) {
        V a[U][8];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = base + u * 64 * VN;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (k < nr && c < lda) a[u][k] = *reinterpret_cast<const V *>(A + (size_t)k * lda + c);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = base + u * 64 * VN;
            if (c < lda) {
                T xv[VN];
#pragma unroll
                for (int v = 0; v < VN; ++v) xv[v] = x[c + v];
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (k < nr)
#pragma unroll
                        for (int v = 0; v < VN; ++v) acc[k] += VT::at(a[u][k], v) * xv[v];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) out[k] = wave_sum(acc[k]);
}

// steps per pass of wave_rows8 (16-byte loads in flight per lane and row)
template <typename T>
constexpr int rows_unroll() {
    return 2;
}

// AND of the class flags of the 64 x 8 blocks that make up the tile of TYv
// rows at (i0, j0); rows beyond the grid count as blocks with no cells.
template <int TYv>
__device__ __forceinline__ unsigned tile_flags(const LevelArgs &L, int i0, int j0) {
    unsigned f = 0xffu;
#pragma unroll
    for (int q = 0; q < TYv / 8; ++q) {
        const int by = (j0 >> 3) + q;
        f &= by < L.full_by ? (unsigned)L.full[by * L.full_bx + (i0 >> 6)] : (unsigned)(FULL_NO_SFV | FULL_DEAD);
    }
    return f;
}

// ---------------------------------------------------------------------------
// Launch A, tile role: weighted Jacobi on the SFV cells, eq. (5.5),
// D = -5(a+c)/(2h^2).  uzero: the old iterate is zero (first sweep of a
// residual equation), so it is not read.
template <typename T, bool MIXED, int TYv>
__device__ __forceinline__ void jacobi_tile(const LevelArgs &L, const T *__restrict__ uold, const T *__restrict__ b,
                                            T *__restrict__ unew, const uint8_t *__restrict__ mask, bool uzero,
                                            int i0, int j0, T (*s)[HX], double *gws) {
    constexpr int R = TYv / (NT / TX);           // consecutive rows per thread
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int i = i0 + tx, r0 = ty * R;
    // a tile with no SFV cell has nothing to update; one made of blocks whose
    // cells are all SFV cells skips the class bytes (TYv is a multiple of 8,
    // i0 of 64, j0 of TYv)
    const unsigned tf = tile_flags<TYv>(L, i0, j0);
    if (tf & FULL_NO_SFV) return;
    const bool full = (tf & FULL_ALL_SFV) != 0;
    // the per-cell loads are issued before the tile barrier so that their
    // latency overlaps the tile load
    uint8_t mk[R];
    T bv[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int j = j0 + r0 + k;
        const bool in = i < L.nx && j < L.ny;
        const size_t id = pidx(L, in ? i : 0, in ? j : 0);
        mk[k] = full ? (uint8_t)1 : (in ? mask[id] : (uint8_t)0);
        bv[k] = b[id];
    }
    const T wod = (T)L.omega_over_d;
    if (uzero) {
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (mk[k] == 1) unew[pidx(L, i, j0 + r0 + k)] = wod * bv[k];
        return;
    }
    auto uat = [&](int a, int c) { return uold[pidx(L, a, c)]; };
    load_tile<T, decltype(uat), TYv>(s, gws, uat, L, i0, j0);
    __syncthreads();
    // a 5 x 5 window of the tile slides down the thread's column: one new
    // row of 5 LDS values per cell instead of the whole stencil
    const int lx = tx + 2;
    T w[5][5];
#pragma unroll
    for (int a = 1; a < 5; ++a)
#pragma unroll
        for (int c = 0; c < 5; ++c) w[a][c] = s[r0 + a - 1][lx - 2 + c];
#pragma unroll
    for (int k = 0; k < R; ++k) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 5; ++c) w[a][c] = w[a + 1][c];
#pragma unroll
        for (int c = 0; c < 5; ++c) w[4][c] = s[r0 + k + 4][lx - 2 + c];
        if (mk[k] != 1) continue;
        T au = apply_sfv<T, MIXED>(L, [&](int dx, int dy) { return w[dy + 2][dx + 2]; });
        unew[pidx(L, i, j0 + r0 + k)] = w[2][2] + wod * (bv[k] - au);
    }
}

// Launch A, tile role of the multicolour variant (an extension of eq.
// (5.5)): the tile with its halo is loaded into LDS from the old iterate
// (ghosts included), then the SFV cells are updated colour by colour in LDS,
// each colour from the values the previous colours left.  Colours: (i + j)
// mod 3 for the plus-shaped stencil, (i + 3 j) mod 9 for the 5 x 5 box, so
// that no two cells of one colour are in each other's stencil and a colour
// is updated in place without races.  Cells in other tiles keep their old
// values for the whole launch (Jacobi across tiles).  In each colour pass
// the threads take consecutive cells of that colour, so every lane works.
template <typename T, bool MIXED, int TYv>
__device__ __forceinline__ void multicolour_tile(const LevelArgs &L, const T *__restrict__ uold,
                                                 const T *__restrict__ b, T *__restrict__ unew,
                                                 const uint8_t *__restrict__ mask, bool uzero, int i0, int j0,
                                                 T (*s)[HX], T (*bs)[TX], uint8_t (*ms)[TX], double *gws) {
    constexpr int NC = MIXED ? 9 : 3, MULT = MIXED ? 3 : 1;
    constexpr int PER_ROW = (TX + NC - 1) / NC;          // cells of one colour per tile row, at most
    constexpr int R = TYv / (NT / TX);
    if (tile_flags<TYv>(L, i0, j0) & FULL_NO_SFV) return;      // nothing to update
    // b and the class bytes of the tile, row-coalesced, into LDS
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int gi = i0 + tx;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = ty * R + k, gj = j0 + r;
        const bool in = gi < L.nx && gj < L.ny;
        const size_t id = pidx(L, in ? gi : 0, in ? gj : 0);
        ms[r][tx] = in ? mask[id] : (uint8_t)0;
        bs[r][tx] = b[id];
    }
    auto uat = [&](int a, int c) { return uzero ? (T)0 : uold[pidx(L, a, c)]; };
    load_tile<T, decltype(uat), TYv>(s, gws, uat, L, i0, j0);
    __syncthreads();
    const T wod = (T)L.omega_over_d;
    for (int k = 0; k < NC; ++k) {
        for (int q = threadIdx.x; q < TYv * PER_ROW; q += NT) {
            const int r = q / PER_ROW, m = q - r * PER_ROW;
            int c0 = (k - i0 - MULT * (j0 + r)) % NC;
            if (c0 < 0) c0 += NC;
            const int lx = c0 + NC * m;
            if (lx >= TX || ms[r][lx] != 1) continue;
            const int ly = r + 2, cx = lx + 2;
            const T au = apply_sfv<T, MIXED>(L, [&](int dx, int dy) { return s[ly + dy][cx + dx]; });
            s[ly][cx] += wod * (bs[r][lx] - au);
        }
        __syncthreads();
    }
    // the updated SFV cells, row-coalesced
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = ty * R + k, gj = j0 + r;
        if (ms[r][tx] == 1) unew[pidx(L, gi, gj)] = s[r + 2][tx + 2];
    }
}

// Launch A, PLG role: one group of PLG rows (a segment slice, or a run of
// separator rows).  Dense row-major blocks are applied one wavefront per
// row, 8 rows at a time: the 64 lanes read consecutive columns and the
// partial sums are reduced across the wavefront.  HNEW: the tile role has
// already run (an earlier launch on the same stream), so the Jacobi-updated
// SFV values are read from unew instead of being recomputed.
template <typename T, bool MIXED, bool HNEW, bool PRE>
__device__ __forceinline__ void plg_group(const LevelArgs &L, const T *__restrict__ uold, const T *__restrict__ b,
                                          T *__restrict__ unew, bool uzero, const PlgDev<T> &P, int bi, T *lds) {
    const PlgBlkA bk = P.blk1[bi];
    const int g = bk.g, r0 = bk.r0, r1 = bk.r1, gs = bk.gs, n = bk.n;
    T *hv = lds, *tt = lds + PLG_HMAX, *yy = tt + PLG_LMAX;     // yy: PLG_SLICE rows
    const T wod = (T)L.omega_over_d;
    // b2 of this thread's rows and this block's entries of A_SB, loaded
    // before the gather
    constexpr int RPT = (PLG_LMAX + NT - 1) / NT;
    T brow[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int q = threadIdx.x + k * NT;
        brow[k] = q < n ? b[P.cell[gs + q]] : (T)0;
    }
    const int ce = bk.ce0 + threadIdx.x;
    int ce_row = -1, ce_slot = 0;
    T ce_val = 0;
    if (ce < bk.ce1) {
        ce_row = P.ce_row[ce];
        ce_slot = P.ce_slot[ce];
        ce_val = P.ce_val[ce];
    }
    // the cell of this thread's output row (levels without separators)
    const int out_cell = (P.nsep == 0 && g < P.nseg && (int)threadIdx.x < r1 - r0) ? P.cell[r0 + threadIdx.x] : 0;
    // PRE (the fused launch on small grids, where the gather below is long:
    // it recomputes the Jacobi update of every coupled SFV cell, and few
    // blocks are resident): this thread's first row of A21 is loaded before
    // the gather, so that its latency overlaps it
    static_assert(!(PRE && HNEW), "the preload serves the fused launch");
    T a0v[PRE ? ELL_W : 1];
    int a0l[PRE ? ELL_W : 1];
    if (PRE && n > 0) {
        const size_t e0 = (size_t)(gs + min((int)threadIdx.x, n - 1)) * ELL_W;
#pragma unroll
        for (int e = 0; e < (PRE ? ELL_W : 1); ++e) {
            a0v[e] = P.a21_val[e0 + e];
            a0l[e] = P.a21_loc[e0 + e];
        }
    }
    // u1 after the Jacobi sweep on the SFV cells the group couples to
    for (int k = threadIdx.x; k < bk.nh; k += NT) {
        const int id = P.hcell[bk.h0 + k];
        T v;
        if (HNEW) {
            v = unew[id];
        } else if (uzero) {
            v = wod * b[id];
        } else {
            const int j = id / L.pitch - 2, i = id - (j + 2) * L.pitch - 2;
            v = uold[id] + wod * (b[id] - sfv_global<T, MIXED>(L, uold, i, j));
        }
        hv[k] = v;
    }
    if (bk.nh == 0 && threadIdx.x == 0) hv[0] = 0;   // target of the zero padding
    __syncthreads();
    // t = b2 - A21 u1
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int q = threadIdx.x + k * NT;
        if (q < n) {
            T v = 0;
            if (PRE && k == 0) {
#pragma unroll
                for (int e = 0; e < (PRE ? ELL_W : 1); ++e) v += a0v[e] * hv[a0l[e]];
            } else {
                const size_t e0 = (size_t)(gs + q) * ELL_W;
#pragma unroll
                for (int e = 0; e < ELL_W; ++e) v += P.a21_val[e0 + e] * hv[P.a21_loc[e0 + e]];
            }
            tt[q] = brow[k] - v;
        }
    }
    const int npad = (n + 3) & ~3;
    if (threadIdx.x < npad - n) tt[n + threadIdx.x] = 0;
    __syncthreads();
    if (g >= P.nseg) {                           // separator rows: right-hand side only
        for (int q = threadIdx.x; q < n; q += NT) P.t[gs + q] = tt[q];
        return;
    }
    // y = B^{-1} t on rows [r0, r1) (row stride npad)
    const T *inv = P.inv + bk.inv_off;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nr = r1 - r0, lr0 = r0 - gs;
    for (int rb = wave * 8; rb < nr; rb += 32) {
        T out[8];
        wave_rows8<T, rows_unroll<T>()>(inv + (size_t)(lr0 + rb) * npad, npad, min(8, nr - rb), tt, lane, out);
        if (lane == 0)
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (rb + k < nr) yy[rb + k] = out[k];
    }
    __syncthreads();
    if (P.nsep == 0) {
        if ((int)threadIdx.x < nr) unew[out_cell] = yy[threadIdx.x];      // nr <= PLG_SLICE <= NT
        return;
    }
    for (int q = threadIdx.x; q < nr; q += NT) P.y[r0 + q] = yy[q];
    // entries of A_SB y on these rows (summed per separator row in launch B)
    if (ce_row >= r0 && ce_row < r1) P.contrib[ce_slot] = ce_val * yy[ce_row - r0];
    for (int k = bk.ce0 + NT + threadIdx.x; k < bk.ce1; k += NT) {
        const int row = P.ce_row[k];
        if (row >= r0 && row < r1) P.contrib[P.ce_slot[k]] = P.ce_val[k] * yy[row - r0];
    }
}

template <typename T, int TYv>
constexpr size_t smooth_a_lds() {
    return sizeof(T) * ((size_t)(TYv + 4) * HX > (size_t)(PLG_HMAX + PLG_LMAX + PLG_SLICE)
                            ? (size_t)(TYv + 4) * HX
                            : (size_t)(PLG_HMAX + PLG_LMAX + PLG_SLICE));
}

// tile heights of launch A: short tiles on small grids (more blocks, shorter
// per-thread chains), tall tiles on large grids (less halo traffic)
constexpr int TY_SMALL = 8;

// Tile of block bid in a launch whose first n blocks are tiles.  Blocks are
// dealt to the 8 XCDs in turn (block b to XCD b mod 8), so this hands each
// XCD a run of consecutive tiles: neighbouring tiles then share the cache
// lines of their common halo in one L2.
__device__ __forceinline__ int xcd_tile(int bid, int n) {
    const int x = bid & 7, k = bid >> 3, q = n >> 3, r = n & 7;
    return x * q + min(x, r) + k;
}

// Block order of launch A.  In FP32 the tiles come first.  In FP64 fewer
// blocks are resident at once, so the PLG blocks (the longer dependency
// chains) come first to start early; their section is padded to a multiple
// of 8 blocks so that the tiles keep their XCD-aligned order.
template <typename T>
constexpr bool plg_first() {
    return sizeof(T) == 8;
}
template <typename T>
__host__ __device__ __forceinline__ int plg_section(int nblk1) {
    return plg_first<T>() ? (nblk1 + 7) & ~7 : nblk1;
}

template <typename T, bool MIXED, int TYv, bool HNEW = false>
__global__ __launch_bounds__(NT) void k_smooth_a(LevelArgs L, const T *__restrict__ uold, const T *__restrict__ b,
                                                 T *__restrict__ unew, const uint8_t *__restrict__ mask, int tiles_x,
                                                 int ntile, int uzero, PlgDev<T> P) {
    __shared__ __align__(16) unsigned char smem[smooth_a_lds<T, TYv>()];
    __shared__ double gws[32];
    const int bid = blockIdx.x;
    const int tile0 = plg_first<T>() ? plg_section<T>(P.nblk1) : 0;         // first tile block
    const int plg0 = plg_first<T>() ? 0 : ntile;                             // first PLG block
    if (bid >= tile0 && bid < tile0 + ntile) {
        const int t = xcd_tile(bid - tile0, ntile);
        jacobi_tile<T, MIXED, TYv>(L, uold, b, unew, mask, uzero != 0, (t % tiles_x) * TX, (t / tiles_x) * TYv,
                                   reinterpret_cast<T(*)[HX]>(smem), gws);
        return;
    }
    if (bid - plg0 >= P.nblk1) return;                                       // padding of the PLG section
    plg_group<T, MIXED, HNEW, !HNEW && TYv == TY_SMALL>(L, uold, b, unew, uzero != 0, P,
                                                        xcd_tile(bid - plg0, P.nblk1), reinterpret_cast<T *>(smem));
}

// Launch A on large grids, tile role alone: it needs far fewer registers
// than the PLG role (about 55 against 145 VGPRs in FP32), so a kernel of its
// own keeps more waves per SIMD in flight to cover the memory latency; the
// PLG groups follow as k_smooth_a with no tiles, reading the SFV values the
// tiles wrote.
// tile height of k_smooth_tiles (the shorter FP64 tiles need fewer registers)
template <typename T>
constexpr int ty_split() {
    return split_tile_rows((int)sizeof(T));
}

template <typename T, bool MIXED, int TYv>
__global__ __launch_bounds__(NT) void k_smooth_tiles(LevelArgs L, const T *__restrict__ uold,
                                                     const T *__restrict__ b, T *__restrict__ unew,
                                                     const uint8_t *__restrict__ mask, int tiles_x, int uzero,
                                                     const int *__restrict__ list) {
    __shared__ __align__(16) T smem[(TYv + 4) * HX];
    __shared__ double gws[32];
    const int k = xcd_tile(blockIdx.x, gridDim.x);
    const int t = list ? list[k] : k;
    jacobi_tile<T, MIXED, TYv>(L, uold, b, unew, mask, uzero != 0, (t % tiles_x) * TX, (t / tiles_x) * TYv,
                               reinterpret_cast<T(*)[HX]>(smem), gws);
}

// Two consecutive sweeps of eq. (5.5) on a tile in one pass, for tiles whose
// cells and 2-cell halo are all SFV cells and whose 4-cell halo lies inside
// the box: the halo's first-sweep values need only old values (no PLG cell
// and no ghost among them), so the tile's second-sweep values follow from
// the first without the PLG block solve in between.  The arithmetic of each
// cell's update is that of jacobi_tile.  The first sweep's values of the
// tile go to ub (the PLG groups and the neighbouring tiles read them), the
// second sweep's to uc.  E2: the tile with its 4-cell halo (old values); E1:
// the tile with its 2-cell halo (first-sweep values).
constexpr int PX = TX + 8;
template <typename T, bool MIXED, int TYv>
__device__ __forceinline__ void pair_tile(const LevelArgs &L, const T *__restrict__ uold, const T *__restrict__ b,
                                          T *__restrict__ ub, T *__restrict__ uc, bool uzero, int i0, int j0,
                                          T (*s2)[PX], T (*s1)[HX]) {
    constexpr int E1 = TYv + 4, RR = (E1 + 3) / 4, R = TYv / 4, NX1 = 4 * E1;
    static_assert(NT == 4 * TX, "four thread rows of 64 columns");
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const T wod = (T)L.omega_over_d;
    // right-hand sides: E1's 64 middle columns (RR rows per thread row) and
    // its 4 outer columns (one cell per thread); the second sweep takes the
    // tile's from LDS
    T b1[RR], bx = 0;
#pragma unroll
    for (int k = 0; k < RR; ++k) {
        const int er = ty * RR + k;
        b1[k] = er < E1 ? b[pidx(L, i0 + tx, j0 - 2 + er)] : (T)0;
    }
    const int xc = threadIdx.x / E1, xr = threadIdx.x - xc * E1;      // outer column xc (0..3), row xr
    const int xe = xc < 2 ? xc : TX + xc;                               // its E1 column
    if (threadIdx.x < NX1) bx = b[pidx(L, i0 - 2 + xe, j0 - 2 + xr)];
    if (!uzero) {
        constexpr int N2 = (TYv + 8) * PX, NL = (N2 + NT - 1) / NT;
        T v[NL];
        // (32-bit offsets from the tile's E2 corner: the arrays of a level
        // hold fewer than 2^31 cells)
        const T *e2 = uold + pidx(L, i0 - 4, j0 - 4);
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int t = min((int)threadIdx.x + k * NT, N2 - 1);
            const int r = t / PX, c = t - r * PX;
            v[k] = e2[(unsigned)(r * L.pitch + c)];
        }
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int t = threadIdx.x + k * NT;
            if (t < N2) s2[t / PX][t % PX] = v[k];
        }
        __syncthreads();
    }
    // first sweep on E1
    if (uzero) {
#pragma unroll
        for (int k = 0; k < RR; ++k) {
            const int er = ty * RR + k;
            if (er < E1) s1[er][tx + 2] = wod * b1[k];
        }
        if (threadIdx.x < NX1) s1[xr][xe] = wod * bx;
    } else {
        T w[5][5];
#pragma unroll
        for (int a = 1; a < 5; ++a)
#pragma unroll
            for (int c = 0; c < 5; ++c) w[a][c] = s2[ty * RR + a - 1][tx + 2 + c];
#pragma unroll
        for (int k = 0; k < RR; ++k) {
            const int er = ty * RR + k;
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 5; ++c) w[a][c] = w[a + 1][c];
            if (er >= E1) break;
#pragma unroll
            for (int c = 0; c < 5; ++c) w[4][c] = s2[er + 4][tx + 2 + c];
            const T au = apply_sfv<T, MIXED>(L, [&](int dx, int dy) { return w[dy + 2][dx + 2]; });
            s1[er][tx + 2] = w[2][2] + wod * (b1[k] - au);
        }
        if (threadIdx.x < NX1) {
            const int ly = xr + 2, lx = xe + 2;
            const T au = apply_sfv<T, MIXED>(L, [&](int dx, int dy) { return s2[ly + dy][lx + dx]; });
            s1[xr][xe] = s2[ly][lx] + wod * (bx - au);
        }
    }
    __syncthreads();
    // the tile's right-hand side into the space of E2, which is no longer
    // read (rows 2 .. TYv+1 of E1 are the tile's rows)
    static_assert(TYv * TX <= (TYv + 8) * PX, "the tile's b fits in E2's space");
    T (*bt)[TX] = reinterpret_cast<T(*)[TX]>(&s2[0][0]);
#pragma unroll
    for (int k = 0; k < RR; ++k) {
        const int er = ty * RR + k;
        if (er >= 2 && er < TYv + 2) bt[er - 2][tx] = b1[k];
    }
    __syncthreads();
    // second sweep on the tile
    const int r0 = ty * R;
    T w[5][5];
#pragma unroll
    for (int a = 1; a < 5; ++a)
#pragma unroll
        for (int c = 0; c < 5; ++c) w[a][c] = s1[r0 + a - 1][tx + c];
#pragma unroll
    for (int k = 0; k < R; ++k) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 5; ++c) w[a][c] = w[a + 1][c];
#pragma unroll
        for (int c = 0; c < 5; ++c) w[4][c] = s1[r0 + k + 4][tx + c];
        const T au = apply_sfv<T, MIXED>(L, [&](int dx, int dy) { return w[dy + 2][dx + 2]; });
        const size_t id = pidx(L, i0 + tx, j0 + r0 + k);
        ub[id] = w[2][2];
        uc[id] = w[2][2] + wod * (bt[r0 + k][tx] - au);
    }
}

// Launch of the first sweep of a pair on a level with two-sweep tiles:
// blocks [0, npad) take the two-sweep tiles (list pairs, padded to a
// multiple of 8 blocks so that the other role keeps its XCD-aligned order),
// the rest the other tiles with SFV cells (list singles), which do the first
// sweep alone into ub; tiles without SFV cells are not launched.
template <typename T, bool MIXED, int TYv>
__global__ __launch_bounds__(NT) void k_smooth_pair(LevelArgs L, const T *__restrict__ uold,
                                                    const T *__restrict__ b, T *__restrict__ ub, T *__restrict__ uc,
                                                    const uint8_t *__restrict__ mask, int tiles_x, int uzero,
                                                    const int *__restrict__ pairs, int npair, int npad,
                                                    const int *__restrict__ singles, int nsingle) {
    __shared__ __align__(16) T s2[(TYv + 8) * PX];
    __shared__ __align__(16) T s1[(TYv + 4) * HX];
    __shared__ double gws[32];
    const int bid = blockIdx.x;
    if (bid < npad) {
        const int k = xcd_tile(bid, npad);
        if (k >= npair) return;
        const int t = pairs[k];
        pair_tile<T, MIXED, TYv>(L, uold, b, ub, uc, uzero != 0, (t % tiles_x) * TX, (t / tiles_x) * TYv,
                                 reinterpret_cast<T(*)[PX]>(s2), reinterpret_cast<T(*)[HX]>(s1));
        return;
    }
    const int t = singles[xcd_tile(bid - npad, nsingle)];
    jacobi_tile<T, MIXED, TYv>(L, uold, b, ub, mask, uzero != 0, (t % tiles_x) * TX, (t / tiles_x) * TYv,
                               reinterpret_cast<T(*)[HX]>(s1), gws);
}

template <typename T, bool MIXED, int TYv>
__global__ __launch_bounds__(NT) void k_smooth_tiles_mc(LevelArgs L, const T *__restrict__ uold,
                                                        const T *__restrict__ b, T *__restrict__ unew,
                                                        const uint8_t *__restrict__ mask, int tiles_x, int uzero) {
    __shared__ __align__(16) T smem[(TYv + 4) * HX];
    __shared__ __align__(16) T bsm[TYv * TX];
    __shared__ uint8_t msm[TYv * TX];
    __shared__ double gws[32];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    multicolour_tile<T, MIXED, TYv>(L, uold, b, unew, mask, uzero != 0, (t % tiles_x) * TX, (t / tiles_x) * TYv,
                                    reinterpret_cast<T(*)[HX]>(smem), reinterpret_cast<T(*)[TX]>(bsm),
                                    reinterpret_cast<uint8_t(*)[TX]>(msm), gws);
}

// Launch B: r_S = t_S - A_SB y (every block forms all of it in LDS), then
// either x_S = S'^{-1} r_S on a run of separator rows, or, for a segment
// slice, x_S on the segment's separator columns and x_B = y - F_j x_S.
// MODE 0 runs all blocks; on levels with many separators launch B is split:
// MODE 1 runs the separator-row blocks (x_S into u), then MODE 2 the segment
// slices, which read their x_S columns from u instead of forming r_S and
// re-reading rows of S'^{-1} slice by slice.
template <typename T, int MODE>
__global__ __launch_bounds__(NT) void k_smooth_b(PlgDev<T> P, T *__restrict__ u) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int ns = P.nsep, nsp = (ns + 3) & ~3;          // dense rows have stride nsp
    T *rs = reinterpret_cast<T *>(smem_raw);
    T *xk = MODE == 2 ? rs : rs + nsp;                  // MODE 2 holds only x_S's columns
    const PlgBlkB bk = P.blk2[xcd_tile(blockIdx.x, gridDim.x) + (MODE == 1 ? P.nblk2_seg : 0)];
    const bool seprows = bk.kind == 1;
    // segment slice: this thread's row of F_j^T and y, loaded before the
    // separator solve (one row per thread: slices have at most NT rows)
    constexpr int KU = 32;                               // columns of F_j held in registers
    const int r = bk.r0 + threadIdx.x;
    const bool myrow = !seprows && r < bk.r1;
    T fv[KU], yr = 0;
    int cr = 0;
    if (myrow) {
        const T *f = P.FT + bk.ft_off + (r - bk.s0);
#pragma unroll
        for (int kk = 0; kk < KU; ++kk) fv[kk] = kk < bk.kj ? f[(size_t)kk * bk.Lj] : (T)0;
        yr = P.y[r];
        cr = P.cell[r];
    }
    // the cells of a separator block's output rows, loaded before the barrier
    __shared__ int ocell[PLG_SEP_ROWS];
    if (MODE != 2 && seprows && (int)threadIdx.x < bk.r1 - bk.r0)
        ocell[threadIdx.x] = P.cell[P.sep_begin + bk.r0 + threadIdx.x];
    if (MODE == 2) {
        const int *fc = P.fcols + P.fcols_ptr[bk.j];
        for (int kk = threadIdx.x; kk < bk.kj; kk += NT) xk[kk] = u[P.cell[P.sep_begin + fc[kk]]];
    }
    for (int s = threadIdx.x; MODE != 2 && s < nsp; s += NT) {
        T v = 0;
        if (s < ns) {
            v = P.t[P.sep_begin + s];
#pragma unroll
            for (int k = 0; k < ELL_W; ++k) v -= P.contrib[(size_t)s * ELL_W + k];
        }
        rs[s] = v;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // dense rows times r_S: rows of S'^{-1} (separator block), or the rows
    // of S'^{-1} at the segment's separator columns
    const T *A = seprows ? P.sinv + (size_t)bk.r0 * nsp : P.SJ + bk.sj_off;
    const int nr = MODE == 2 ? 0 : seprows ? bk.r1 - bk.r0 : bk.kj;
    for (int rb = wave * 8; rb < nr; rb += 32) {
        T out[8];
        wave_rows8<T, rows_unroll<T>()>(A + (size_t)rb * nsp, nsp, min(8, nr - rb), rs, lane, out);
        if (lane == 0)
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (rb + k < nr) {
                    if (seprows) u[ocell[rb + k]] = out[k];
                    else xk[rb + k] = out[k];
                }
    }
    if (seprows) return;
    __syncthreads();
    if (!myrow) return;
    const int kj = bk.kj;
    T v0 = 0, v1 = 0, v2 = 0, v3 = 0;
#pragma unroll
    for (int kk = 0; kk < KU; kk += 4) {
        if (kk < kj) v0 += fv[kk] * xk[kk];
        if (kk + 1 < kj) v1 += fv[kk + 1] * xk[kk + 1];
        if (kk + 2 < kj) v2 += fv[kk + 2] * xk[kk + 2];
        if (kk + 3 < kj) v3 += fv[kk + 3] * xk[kk + 3];
    }
    const T *f = P.FT + bk.ft_off + (r - bk.s0);
    for (int kk = KU; kk < kj; ++kk) v0 += f[(size_t)kk * bk.Lj] * xk[kk];
    u[cr] = yr - ((v0 + v1) + (v2 + v3));
}

// ---------------------------------------------------------------------------
// residual of the PLG rows (all columns), solve order
template <typename T>
__global__ void k_plg_residual(int m, const int *__restrict__ cell, const int *__restrict__ ptr,
                               const int *__restrict__ col, const T *__restrict__ val, const T *__restrict__ b,
                               const T *__restrict__ u, T *__restrict__ r) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    T v = b[cell[q]];
    for (int e = ptr[q]; e < ptr[q + 1]; ++e) v -= val[e] * u[col[e]];
    r[q] = v;
}

// Residual of the fine level fused with the restriction of eq. (5.8) (RESID;
// else the restriction of b itself, as FMG restricts residuals): one thread
// per coarse cell, children summed with weight 1/4.  Fine PLG cells
// contribute rplg, or 0 when rplg is null (after a block-smoother sweep the
// PLG rows are solved exactly, Definition 5.6).  rmask (coarse level): 0
// inactive (b = 0), 1 regular, 2 a cell that also absorbs fine cells of a
// merged-away coarse cell, computed by the extra blocks after the tiles,
// one thread per such cell over its list of children.  uc (optional) is the
// coarse iterate, set to zero.
template <typename T, bool MIXED, bool RESID>
__global__ __launch_bounds__(NT) void k_restrict(LevelArgs L, LevelArgs C, int tiles_x, int ntile,
                                                 const T *__restrict__ u, const T *__restrict__ b,
                                                 const uint8_t *__restrict__ mask, const int *__restrict__ plgidx,
                                                 const T *__restrict__ rplg, const uint8_t *__restrict__ rmask,
                                                 T *__restrict__ bc, T *__restrict__ uc, int nt,
                                                 const int *__restrict__ ex_ptr, const int *__restrict__ ex_target,
                                                 const int *__restrict__ ex_child, int skip_dead) {
    __shared__ T s[HY][HX];
    __shared__ double gws[32];
    if ((int)blockIdx.x >= ntile) {
        const int t = (blockIdx.x - ntile) * NT + threadIdx.x;
        if (t >= nt) return;
        T sum = 0;
        for (int e = ex_ptr[t]; e < ex_ptr[t + 1]; ++e) {
            const int id = ex_child[e];
            const int j = id / L.pitch - 2, i = id - (j + 2) * L.pitch - 2;
            if (!RESID)
                sum += mask[id] ? b[id] : (T)0;
            else if (mask[id] == 1)
                sum += b[id] - sfv_global<T, MIXED>(L, u, i, j);
            else if (mask[id] == 2 && rplg)
                sum += rplg[plgidx[id]];
        }
        bc[ex_target[t]] = (T)0.25 * sum;
        if (uc) uc[ex_target[t]] = 0;
        return;
    }
    // the tile's fine cells: each thread owns R consecutive rows of one
    // column and slides a 5 x 5 window down it (as in the smoother); each
    // pair of rows is summed as it completes, then across the neighbouring
    // lane, and the even lanes write the coarse cells
    // with skip_dead the launch covers the listed tiles only (a tile with no
    // active cell over inactive coarse cells would write zeros over zeros)
    const int tk = xcd_tile(blockIdx.x, ntile);
    const int tile = skip_dead ? L.live[tk] : tk;
    const int i0 = (tile % tiles_x) * TX, j0 = (tile / tiles_x) * TY;
    constexpr int R = TY / (NT / TX);
    static_assert(R % 2 == 0, "rows per thread come in pairs");
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int i = i0 + tx, r0 = ty * R;
    const bool col_in = i < L.nx;
    const bool full = (tile_flags<TY>(L, i0, j0) & FULL_ALL_SFV) != 0;
    uint8_t mk[R];
    T bv[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int j = j0 + r0 + k;
        const bool in = col_in && j < L.ny;
        const size_t id = pidx(L, in ? i : 0, in ? j : 0);
        mk[k] = full ? (uint8_t)1 : in ? mask[id] : (uint8_t)0;
        bv[k] = b[id];
    }
    // the residuals of this thread's PLG cells, loaded before the tile
    // barrier (they overwrite bv)
    if (RESID && !full) {
        int pq[R];
#pragma unroll
        for (int k = 0; k < R; ++k) pq[k] = (mk[k] == 2 && rplg) ? plgidx[pidx(L, i, j0 + r0 + k)] : -1;
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (pq[k] >= 0) bv[k] = rplg[pq[k]];
    }
    const int ci = i >> 1;
    // row pair (k - 1, k) complete: sum across the lane pair, even lanes write
    auto emit = [&](int k, T pair) {
        const T other = __shfl_xor(pair, 1, 64);
        const int cj = (j0 + r0 + k) >> 1;
        if ((tx & 1) || ci >= C.nx || cj >= C.ny) return;
        const size_t cid = pidx(C, ci, cj);
        const uint8_t ck = rmask[cid];
        if (ck == 2) return;                        // cells with extra children: the list blocks
        if (uc) uc[cid] = 0;
        bc[cid] = ck ? (T)0.25 * (pair + other) : (T)0;
    };
    if (RESID) {
        load_tile<T>(s, gws, [&](int a, int c) { return u[pidx(L, a, c)]; }, L, i0, j0);
        __syncthreads();
        const int lx = tx + 2;
        T w[5][5];
#pragma unroll
        for (int a = 1; a < 5; ++a)
#pragma unroll
            for (int c = 0; c < 5; ++c) w[a][c] = s[r0 + a - 1][lx - 2 + c];
        T pair = 0;
#pragma unroll
        for (int k = 0; k < R; ++k) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 5; ++c) w[a][c] = w[a + 1][c];
#pragma unroll
            for (int c = 0; c < 5; ++c) w[4][c] = s[r0 + k + 4][lx - 2 + c];
            T r = (T)0;
            if (mk[k] == 1)
                r = bv[k] - apply_sfv<T, MIXED>(L, [&](int dx, int dy) { return w[dy + 2][dx + 2]; });
            else if (mk[k] == 2 && rplg)
                r = bv[k];
            if (k & 1) emit(k - 1, pair + r);
            else pair = r;
        }
    } else {
#pragma unroll
        for (int k = 0; k < R; k += 2)
            emit(k, (mk[k] ? bv[k] : (T)0) + (mk[k + 1] ? bv[k + 1] : (T)0));
    }
}

// Piecewise-constant interpolation and correction, eq. (5.9) (SET: the
// interpolant itself, as FMG starts a V-cycle from it).  Blocks [0, nmain)
// take one coarse cell per thread and its 2 x 2 fine children with one
// 2-element vector access per fine row (the children of a coarse cell start
// at an even padded index); the rest handle the fine cells whose coarse
// parent was merged away (they take the value of the absorbing cell).  A
// coarse cell that is not active leaves its children to those blocks, so
// its thread touches only the inactive children (SET) or nothing.
template <typename T>
struct Vec2;
template <>
struct Vec2<float> { using V = float2; };
template <>
struct Vec2<double> { using V = double2; };

template <typename T, bool SET>
__global__ __launch_bounds__(256) void k_prolong(LevelArgs L, LevelArgs C, int nmain,
                                                 const uint8_t *__restrict__ mask, const uint8_t *__restrict__ cmask,
                                                 const T *__restrict__ ec, T *__restrict__ u, int nex,
                                                 const int *__restrict__ ex_fine, const int *__restrict__ ex_coarse) {
    using V = typename Vec2<T>::V;
    if ((int)blockIdx.x >= nmain) {
        const int k = (blockIdx.x - nmain) * blockDim.x + threadIdx.x;
        if (k < nex) {
            if (SET) u[ex_fine[k]] = ec[ex_coarse[k]];
            else u[ex_fine[k]] += ec[ex_coarse[k]];
        }
        return;
    }
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= C.nx * C.ny) return;
    const int cj = t / C.nx, ci = t - cj * C.nx;
    const size_t cid = pidx(C, ci, cj);
    const uint8_t cm = cmask[cid];
    if (!SET && !cm) return;
    const T e = cm ? ec[cid] : (T)0;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const size_t id = pidx(L, 2 * ci, 2 * cj + r);
        const uchar2 m = *reinterpret_cast<const uchar2 *>(mask + id);
        if (!cm) {                                  // SET only: zero the inactive children
            if (!m.x) u[id] = (T)0;
            if (!m.y) u[id + 1] = (T)0;
            continue;
        }
        V v = *reinterpret_cast<const V *>(u + id);
        if (SET) {
            v.x = m.x ? e : (T)0;
            v.y = m.y ? e : (T)0;
        } else {
            if (m.x) v.x += e;
            if (m.y) v.y += e;
        }
        *reinterpret_cast<V *>(u + id) = v;
    }
}

// ---------------------------------------------------------------------------
// Bottom solve x = A_c^{-1} b (FP64 dense inverse, row-major): one wavefront
// per row, 16 wavefronts per block, the right-hand side staged in LDS by
// every block; 4 independent partial sums per lane keep more loads in flight.
constexpr int BOT_WAVES = 16;
template <typename TI, typename TO>
__global__ __launch_bounds__(64 * BOT_WAVES) void k_bottom(int n, const int *__restrict__ cells,
                                                          const double *__restrict__ ainv, const TI *__restrict__ b,
                                                          TO *__restrict__ x) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *bs = reinterpret_cast<double *>(smem_raw);
    for (int k = threadIdx.x; k < n; k += blockDim.x) bs[k] = (double)b[cells[k]];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = blockIdx.x * BOT_WAVES + wave;
    if (row >= n) return;
    const double *a = ainv + (size_t)row * n;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int c = lane;
    for (; c + 192 < n; c += 256) {
        a0 += a[c] * bs[c];
        a1 += a[c + 64] * bs[c + 64];
        a2 += a[c + 128] * bs[c + 128];
        a3 += a[c + 192] * bs[c + 192];
    }
    for (; c < n; c += 64) a0 += a[c] * bs[c];
    const double acc = wave_sum((a0 + a1) + (a2 + a3));
    if (lane == 0) x[cells[row]] = (TO)acc;
}

// ---------------------------------------------------------------------------
// Dense FP64 inverse of the coarsest level's matrix (setup only): Gauss-Jordan
// elimination with partial pivoting on the augmented n x 2n row-major array
// W = [A | I], one pivot column per step, two launches per step.  On exit
// the right half holds A^{-1}.  status != 0 (set by the pivot kernel: the
// 1-based step whose best pivot is below `tiny` or not finite) makes every
// later launch return at once.
__global__ __launch_bounds__(1024) void k_gj_pivot(int n, int k, double *__restrict__ W, double *__restrict__ f,
                                                   int *__restrict__ status, double tiny) {
    __shared__ double vmax[16];
    __shared__ int imax[16];
    __shared__ int piv_row;
    __shared__ double piv_inv;
    if (*status) return;
    const size_t ld = 2 * (size_t)n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double best = -1.0;
    int bi = k;
    for (int i = k + threadIdx.x; i < n; i += blockDim.x) {
        const double v = fabs(W[(size_t)i * ld + k]);
        if (v > best) { best = v; bi = i; }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_down(best, off, 64);
        const int oi = __shfl_down(bi, off, 64);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if (lane == 0) { vmax[wave] = best; imax[wave] = bi; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double bv = vmax[0];
        int b = imax[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
            if (vmax[w] > bv || (vmax[w] == bv && imax[w] < b)) { bv = vmax[w]; b = imax[w]; }
        const bool ok = bv > tiny && bv <= 1.7976931348623157e308;
        if (!ok) *status = k + 1;
        piv_row = ok ? b : -1;
        piv_inv = ok ? 1.0 / W[(size_t)b * ld + k] : 0.0;
    }
    __syncthreads();
    const int p = piv_row;
    if (p < 0) return;
    const double s = piv_inv;
    // swap rows k and p, scale the pivot row (columns below k are zero in
    // both rows' left halves)
    for (size_t j = (size_t)k + threadIdx.x; j < ld; j += blockDim.x) {
        const double vk = W[(size_t)k * ld + j], vp = W[(size_t)p * ld + j];
        W[(size_t)p * ld + j] = vk;
        W[(size_t)k * ld + j] = vp * s;
    }
    __syncthreads();
    // multipliers of the elimination: column k of the other rows
    for (int i = threadIdx.x; i < n; i += blockDim.x) f[i] = i == k ? 0.0 : W[(size_t)i * ld + k];
}

// W[i][j] -= f[i] W[k][j] for rows i != k and columns j >= k; each block
// takes 4 rows and 256 consecutive columns.
__global__ __launch_bounds__(256) void k_gj_eliminate(int n, int k, double *__restrict__ W,
                                                      const double *__restrict__ f, const int *__restrict__ status) {
    if (*status) return;
    const size_t ld = 2 * (size_t)n;
    const size_t j = (size_t)k + (size_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= ld) return;
    const double pk = W[(size_t)k * ld + j];
    for (int r = 0; r < 4; ++r) {
        const int i = blockIdx.y * 4 + r;
        if (i >= n || i == k) continue;
        W[(size_t)i * ld + j] -= f[i] * pk;
    }
}

// ---------------------------------------------------------------------------
// Residual max-norm over the active cells, FP64: tiles compute the SFV rows
// by the stencil; blocks after the tiles compute the PLG rows from their
// fixed-width rows (one thread per row).  CORRECT: the iterate is u + e (e
// the correction of the cycle just run, FP32 or FP64) and the tiles write it
// to uout (a different buffer); WRITE32: the residual is also written in FP32 (the next FP32
// V-cycle's right-hand side).  One partial maximum per block.
template <bool MIXED, bool WRITE32, bool CORRECT, typename TE>
__global__ __launch_bounds__(NT) void k_residual_norm(LevelArgs L, int tiles_x, int ntile, const double *__restrict__ u,
                                                      const TE *__restrict__ e, double *__restrict__ uout,
                                                      const double *__restrict__ b, const uint8_t *__restrict__ mask,
                                                      int m, const int *__restrict__ pcell,
                                                      const int *__restrict__ fe_col,
                                                      const double *__restrict__ fe_val, float *__restrict__ r32,
                                                      double *__restrict__ r64, double *__restrict__ partial) {
    __shared__ double s[HY][HX];
    __shared__ double gws[32];
    __shared__ double red[NT / 64];
    auto uat = [&](size_t id) { return CORRECT ? u[id] + (double)e[id] : u[id]; };
    double mx = 0.0;
    if ((int)blockIdx.x >= ntile) {
        const int q = (blockIdx.x - ntile) * NT + threadIdx.x;
        if (q < m) {
            const int id = pcell[q];
            const size_t e0 = (size_t)q * ELL_W;
            double r = b[id];
#pragma unroll
            for (int f = 0; f < ELL_W; ++f) r -= fe_val[e0 + f] * uat(fe_col[e0 + f]);
            if (WRITE32) r32[id] = (float)r;
            if (r64) r64[id] = r;
            mx = fabs(r);
        }
    } else {
        // without a caller's buffer r64 the launch covers the listed tiles
        // only (a tile with no active cell writes only zeros, which the
        // hierarchy's own buffers already hold there).  Each thread owns R
        // consecutive rows of one column and slides a 5 x 5 window of the
        // tile down it (as in the smoother).
        constexpr int R = TY / (NT / TX);
        const int tk = xcd_tile(blockIdx.x, ntile);
        const int tile = (L.live && !r64) ? L.live[tk] : tk;
        const int i0 = (tile % tiles_x) * TX, j0 = (tile / tiles_x) * TY;
        const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
        const int i = i0 + tx, r0 = ty * R;
        const bool full = (tile_flags<TY>(L, i0, j0) & FULL_ALL_SFV) != 0;
        uint8_t mk[R];
        double bv[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int j = j0 + r0 + k;
            const bool in = i < L.nx && j < L.ny;
            const size_t id = pidx(L, in ? i : 0, in ? j : 0);
            mk[k] = full ? (uint8_t)1 : in ? mask[id] : (uint8_t)0;
            bv[k] = b[id];
        }
        load_tile<double>(s, gws, [&](int a, int c) { return uat(pidx(L, a, c)); }, L, i0, j0);
        __syncthreads();
        double w[5][5];
#pragma unroll
        for (int a = 1; a < 5; ++a)
#pragma unroll
            for (int c = 0; c < 5; ++c) w[a][c] = s[r0 + a - 1][tx + c];
#pragma unroll
        for (int k = 0; k < R; ++k) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 5; ++c) w[a][c] = w[a + 1][c];
#pragma unroll
            for (int c = 0; c < 5; ++c) w[4][c] = s[r0 + k + 4][tx + c];
            const int j = j0 + r0 + k;
            if (i >= L.nx || j >= L.ny) continue;
            const size_t id = pidx(L, i, j);
            if (CORRECT) uout[id] = mk[k] ? w[2][2] : 0.0;
            if (mk[k] == 2) continue;                 // PLG rows: the blocks after the tiles
            double r = 0.0;
            if (mk[k] == 1) r = bv[k] - apply_sfv<double, MIXED>(L, [&](int dx, int dy) { return w[dy + 2][dx + 2]; });
            if (WRITE32) r32[id] = (float)r;
            if (r64) r64[id] = r;
            mx = fmax(mx, fabs(r));
        }
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = red[0];
        for (int w = 1; w < NT / 64; ++w) v = fmax(v, red[w]);
        partial[blockIdx.x] = v;
    }
}

__global__ void k_absmax(int n, const double *__restrict__ v, const uint8_t *__restrict__ mask,
                         double *__restrict__ partial) {
    __shared__ double red[256];
    double mx = 0.0;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
        if (!mask || mask[k]) mx = fmax(mx, fabs(v[k]));
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// b = f - N g (eq. (4.19)) on the finest level
__global__ void k_copy_active(size_t n, const uint8_t *__restrict__ mask, const double *__restrict__ src,
                              double *__restrict__ dst) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = mask[k] ? src[k] : 0.0;
}

__global__ void k_rhs_rows(int nrows, const int *__restrict__ ptr, const int *__restrict__ cell,
                           const int *__restrict__ gidx, const double *__restrict__ coef,
                           const double *__restrict__ g, double *__restrict__ b) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    double s = 0.0;
    for (int e = ptr[r]; e < ptr[r + 1]; ++e) s += coef[e] * g[gidx[e]];
    b[cell[r]] -= s;
}

__global__ void k_zero_inactive(size_t n, const uint8_t *__restrict__ mask, double *__restrict__ u) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n && !mask[k]) u[k] = 0.0;
}

// ---------------------------------------------------------------------------
// K11: weighted minimum-norm fits (eqs. (4.16)-(4.18)), FP64, one thread per
// PLG cell.  With W = diag(1/w_k), beta = W^{1/2} gamma where gamma is the
// minimum-norm solution of (M W^{1/2}) gamma = phibar: Householder QR of
// B = (M W^{1/2})^T = Q R, then R^T z = phibar and gamma = Q [z; 0].
__global__ void k_fit(int m, const double *__restrict__ Mall, const double *__restrict__ phi,
                      const double *__restrict__ wall, const int *__restrict__ ncol, double *__restrict__ work,
                      double *__restrict__ beta, int *__restrict__ status) {
    constexpr int NBv = 15, KMAX = 16;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    const int K = ncol[r];
    const double *M = Mall + (size_t)r * NBv * KMAX;       // column k = M[k*15 + row]
    const double *w = wall + (size_t)r * KMAX;
    double *B = work + (size_t)r * (2 * KMAX * NBv + KMAX + NBv);   // K x 15, column-major: B[c*KMAX + k]
    double *V = B + KMAX * NBv;                                       // reflectors
    double *vn = V + KMAX * NBv;                                      // |v|^2 per column
    double *y = vn + NBv;                                             // length KMAX
    for (int k = 0; k < K; ++k) {
        const double sq = 1.0 / sqrt(w[k]);
        for (int c = 0; c < NBv; ++c) B[c * KMAX + k] = M[k * NBv + c] * sq;
    }
    int ok = 1;
    for (int c = 0; c < NBv; ++c) {
        double nrm = 0.0;
        for (int k = c; k < K; ++k) nrm += B[c * KMAX + k] * B[c * KMAX + k];
        nrm = sqrt(nrm);
        const double x0 = B[c * KMAX + c];
        const double alpha = x0 >= 0.0 ? -nrm : nrm;
        double vv = 0.0;
        for (int k = c; k < K; ++k) {
            const double v = (k == c) ? x0 - alpha : B[c * KMAX + k];
            V[c * KMAX + k] = v;
            vv += v * v;
        }
        vn[c] = vv;
        if (vv > 0.0) {
            for (int c2 = c + 1; c2 < NBv; ++c2) {
                double d = 0.0;
                for (int k = c; k < K; ++k) d += V[c * KMAX + k] * B[c2 * KMAX + k];
                const double f = 2.0 * d / vv;
                for (int k = c; k < K; ++k) B[c2 * KMAX + k] -= f * V[c * KMAX + k];
            }
        }
        B[c * KMAX + c] = alpha;
        if (alpha == 0.0) ok = 0;
    }
    // R^T z = phibar (R upper triangular: R[i][c] = B[c*KMAX + i], i <= c)
    for (int i = 0; i < KMAX; ++i) y[i] = 0.0;
    for (int c = 0; c < NBv && ok; ++c) {
        double s = phi[(size_t)r * NBv + c];
        for (int i = 0; i < c; ++i) s -= B[c * KMAX + i] * y[i];
        y[c] = s / B[c * KMAX + c];
    }
    // gamma = H_0 H_1 ... H_14 [z; 0]
    for (int c = NBv - 1; c >= 0; --c) {
        if (vn[c] == 0.0) continue;
        double d = 0.0;
        for (int k = c; k < K; ++k) d += V[c * KMAX + k] * y[k];
        const double f = 2.0 * d / vn[c];
        for (int k = c; k < K; ++k) y[k] -= f * V[c * KMAX + k];
    }
    for (int k = 0; k < K; ++k) beta[(size_t)r * KMAX + k] = y[k] / sqrt(w[k]);
    status[r] = ok;
}

// ---------------------------------------------------------------------------
// launchers
namespace {
inline dim3 tile_grid(const LevelArgs &L) { return dim3((L.nx + TX - 1) / TX, (L.ny + TY - 1) / TY); }
}  // namespace

template <typename T>
void launch_smooth_a(const LevelArgs &L, const T *uold, const T *b, T *unew, const uint8_t *mask, bool uzero,
                     const PlgDev<T> &P, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    const bool small = (sizeof(T) == 4 ? L.small32 : L.small64) != 0;
    const int ty = small ? TY_SMALL : TY;
    const int tiles_x = (L.nx + TX - 1) / TX, ntile = tiles_x * ((L.ny + ty - 1) / ty);
    const int uz = uzero ? 1 : 0;
    if (L.colouring) {
        // the PLG groups read the SFV values the tiles wrote (they cannot
        // recompute a multicolour sweep)
        constexpr int tys = ty_split<T>();
        const int nts = tiles_x * ((L.ny + tys - 1) / tys);
        if (L.mixed)
            hipExtLaunchKernelGGL((k_smooth_tiles_mc<T, true, tys>), dim3(nts), dim3(NT), 0, st, ev0, ev1, 0, L,
                                  uold, b, unew, mask, tiles_x, uz);
        else
            hipExtLaunchKernelGGL((k_smooth_tiles_mc<T, false, tys>), dim3(nts), dim3(NT), 0, st, ev0, ev1, 0, L,
                                  uold, b, unew, mask, tiles_x, uz);
        if (P.nblk1 == 0) return;
        hipLaunchKernelGGL((k_smooth_a<T, false, TY, true>), dim3(P.nblk1), dim3(NT), 0, st, L, uold, b, unew,
                           mask, tiles_x, 0, uz, P);
        return;
    }
    if (L.split_a) {
        // the tiles write the SFV cells, then the PLG groups read those
        // of their couplings and write the PLG rows
        constexpr int tys = ty_split<T>();
        const int nts = tiles_x * ((L.ny + tys - 1) / tys);
        if (L.mixed)
            hipExtLaunchKernelGGL((k_smooth_tiles<T, true, tys>), dim3(nts), dim3(NT), 0, st, ev0, ev1, 0, L, uold,
                                  b, unew, mask, tiles_x, uz, (const int *)nullptr);
        else
            hipExtLaunchKernelGGL((k_smooth_tiles<T, false, tys>), dim3(nts), dim3(NT), 0, st, ev0, ev1, 0, L, uold,
                                  b, unew, mask, tiles_x, uz, (const int *)nullptr);
        if (P.nblk1 == 0) return;
        // no stencil is evaluated here, so one instantiation serves b = 0 and b != 0
        hipLaunchKernelGGL((k_smooth_a<T, false, TY, true>), dim3(P.nblk1), dim3(NT), 0, st, L, uold, b, unew,
                           mask, tiles_x, 0, uz, P);
        return;
    }
    const dim3 grid(ntile + plg_section<T>(P.nblk1));
#define MG_SA(MX, TYV)                                                                                           \
    hipExtLaunchKernelGGL((k_smooth_a<T, MX, TYV>), grid, dim3(NT), 0, st, ev0, ev1, 0, L, uold, b, unew, mask, tiles_x, \
                          ntile, uz, P)
    if (L.mixed) { if (small) MG_SA(true, TY_SMALL); else MG_SA(true, TY); }
    else { if (small) MG_SA(false, TY_SMALL); else MG_SA(false, TY); }
#undef MG_SA
}

// Two sweeps on a level whose launch A is split: the first sweep's tiles
// (two-sweep tiles also doing the second) into ub, the PLG groups and launch
// B on ub; the second sweep's remaining tiles from ub into uc, the PLG groups
// and launch B on uc.
template <typename T>
void launch_smooth_pair(const LevelArgs &L, const T *uold, const T *b, T *ub, T *uc, const uint8_t *mask,
                        bool uzero, const PlgDev<T> &P, const int *pairs, int npair, const int *singles, int nsingle,
                        hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    constexpr int tys = ty_split<T>();
    const int tiles_x = (L.nx + TX - 1) / TX;
    const int npad = (npair + 7) & ~7;
    const int uz = uzero ? 1 : 0;
    if (L.mixed)
        hipExtLaunchKernelGGL((k_smooth_pair<T, true, tys>), dim3(npad + nsingle), dim3(NT), 0, st, ev0, ev1, 0, L,
                              uold, b, ub, uc, mask, tiles_x, uz, pairs, npair, npad, singles, nsingle);
    else
        hipExtLaunchKernelGGL((k_smooth_pair<T, false, tys>), dim3(npad + nsingle), dim3(NT), 0, st, ev0, ev1, 0, L,
                              uold, b, ub, uc, mask, tiles_x, uz, pairs, npair, npad, singles, nsingle);
    if (P.nblk1)
        hipLaunchKernelGGL((k_smooth_a<T, false, TY, true>), dim3(P.nblk1), dim3(NT), 0, st, L, uold, b, ub, mask,
                           tiles_x, 0, uz, P);
    launch_smooth_b<T>(P, ub, st);
    if (nsingle) {
        if (L.mixed)
            hipLaunchKernelGGL((k_smooth_tiles<T, true, tys>), dim3(nsingle), dim3(NT), 0, st, L, ub, b, uc, mask,
                               tiles_x, 0, singles);
        else
            hipLaunchKernelGGL((k_smooth_tiles<T, false, tys>), dim3(nsingle), dim3(NT), 0, st, L, ub, b, uc, mask,
                               tiles_x, 0, singles);
    }
    if (P.nblk1)
        hipLaunchKernelGGL((k_smooth_a<T, false, TY, true>), dim3(P.nblk1), dim3(NT), 0, st, L, ub, b, uc, mask,
                           tiles_x, 0, 0, P);
    launch_smooth_b<T>(P, uc, st);
}

template <typename T>
void launch_smooth_b(const PlgDev<T> &P, T *unew, hipStream_t st) {
    if (!P.nblk2) return;
    const size_t lds = sizeof(T) * (((P.nsep + 3) & ~3) + PLG_KMAX);
    if (P.split_b && P.nblk2_seg > 0 && P.nblk2_seg < P.nblk2) {
        hipLaunchKernelGGL((k_smooth_b<T, 1>), dim3(P.nblk2 - P.nblk2_seg), dim3(NT), lds, st, P, unew);
        hipLaunchKernelGGL((k_smooth_b<T, 2>), dim3(P.nblk2_seg), dim3(NT), sizeof(T) * PLG_KMAX, st, P, unew);
        return;
    }
    hipLaunchKernelGGL((k_smooth_b<T, 0>), dim3(P.nblk2), dim3(NT), lds, st, P, unew);
}

template <typename T>
__global__ void k_fill_zero(size_t n, T *__restrict__ u) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) u[k] = (T)0;
}

template <typename T>
void launch_fill_zero(size_t n, T *u, hipStream_t st) {
    hipLaunchKernelGGL((k_fill_zero<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, u);
}


template <typename T>
void launch_plg_residual(int m, const int *cell, const int *ptr, const int *col, const T *val, const T *b,
                         const T *u, T *r, hipStream_t st) {
    if (m == 0) return;
    hipLaunchKernelGGL((k_plg_residual<T>), dim3((m + 255) / 256), dim3(256), 0, st, m, cell, ptr, col, val, b, u, r);
}

template <typename T>
void launch_restrict(const LevelArgs &L, const LevelArgs &C, const T *u, const T *b, const uint8_t *mask,
                     const int *plgidx, const T *rplg, const uint8_t *rmask, T *bc, T *uc, int nt, const int *ex_ptr,
                     const int *ex_target, const int *ex_child, bool skip_dead, hipStream_t st) {
    const int tx = (C.nx + TX / 2 - 1) / (TX / 2), ty = (C.ny + TY / 2 - 1) / (TY / 2);
    // the list numbers the fine level's 64 x 32 tiles, the same tiles when
    // the fine grid is twice the coarse one
    skip_dead = skip_dead && L.live && tx == (L.nx + TX - 1) / TX;
    const int ntile = skip_dead ? L.nlive : tx * ty;
    const dim3 grid(ntile + (nt + NT - 1) / NT);
#define MG_RS(MX, RS)                                                                                            \
    hipLaunchKernelGGL((k_restrict<T, MX, RS>), grid, dim3(NT), 0, st, L, C, tx, ntile, u, b, mask, plgidx, rplg, \
                       rmask, bc, uc, nt, ex_ptr, ex_target, ex_child, skip_dead ? 1 : 0)
    if (!u) MG_RS(false, false);
    else if (L.mixed) MG_RS(true, true);
    else MG_RS(false, true);
#undef MG_RS
}

template <typename T>
void launch_prolong(const LevelArgs &L, const LevelArgs &C, const uint8_t *mask, const uint8_t *cmask, const T *ec,
                    T *u, int nex, const int *ex_fine, const int *ex_coarse, bool set, hipStream_t st) {
    const int nmain = (C.nx * C.ny + 255) / 256;
    const dim3 grid(nmain + (nex + 255) / 256);
    if (set)
        hipLaunchKernelGGL((k_prolong<T, true>), grid, dim3(256), 0, st, L, C, nmain, mask, cmask, ec, u, nex,
                           ex_fine, ex_coarse);
    else
        hipLaunchKernelGGL((k_prolong<T, false>), grid, dim3(256), 0, st, L, C, nmain, mask, cmask, ec, u, nex,
                           ex_fine, ex_coarse);
}

template <typename TI, typename TO>
void launch_bottom(int n, const int *cells, const double *ainv, const TI *b, TO *x, hipStream_t st) {
    hipLaunchKernelGGL((k_bottom<TI, TO>), dim3((n + BOT_WAVES - 1) / BOT_WAVES), dim3(64 * BOT_WAVES),
                       sizeof(double) * n, st, n, cells, ainv, b, x);
}

int launch_residual_norm(const LevelArgs &L, const double *u, const void *e, bool e64, double *uout, const double *b,
                         const uint8_t *mask, int m, const int *pcell, const int *fe_col, const double *fe_val,
                         float *r32, double *r64, double *partial, hipStream_t st) {
    const dim3 tg = tile_grid(L);
    const int ntile = (L.live && !r64) ? L.nlive : (int)(tg.x * tg.y), nblk = ntile + (m + NT - 1) / NT;
#define MG_RES(MX, W32, CORR, TE)                                                                                      \
    hipLaunchKernelGGL((k_residual_norm<MX, W32, CORR, TE>), dim3(nblk), dim3(NT), 0, st, L, (int)tg.x, ntile, u,       \
                       static_cast<const TE *>(e), uout, b, mask, m, pcell, fe_col, fe_val, r32, r64, partial)
#define MG_RES2(MX, W32)                                          \
    if (!e) MG_RES(MX, W32, false, float);                        \
    else if (e64) MG_RES(MX, W32, true, double);                  \
    else MG_RES(MX, W32, true, float);
    const bool w32 = r32 != nullptr;
    if (L.mixed) { if (w32) { MG_RES2(true, true) } else { MG_RES2(true, false) } }
    else { if (w32) { MG_RES2(false, true) } else { MG_RES2(false, false) } }
#undef MG_RES2
#undef MG_RES
    return nblk;
}

int residual_norm_blocks(const LevelArgs &L, int m) {
    const dim3 tg = tile_grid(L);
    return (int)(tg.x * tg.y) + (m + NT - 1) / NT;
}

// Fixed device memory for the entry point that allocates nothing
// (mg_residual_norm_noalloc): the per-block partial maxima of the residual
// norm.  Each device holds its own copy for the life of the process; host
// code must use the address from noalloc_scratch(), never the symbol.
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

double *noalloc_scratch() {
    static std::mutex mu;
    static std::map<int, double *> addr;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) return it->second;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    addr[dev] = (double *)p;
    return (double *)p;
}

void launch_absmax(int n, const double *v, const uint8_t *mask, double *partial, int nblocks, hipStream_t st) {
    hipLaunchKernelGGL(k_absmax, dim3(nblocks), dim3(256), 0, st, n, v, mask, partial);
}

void launch_rhs(size_t n, const uint8_t *mask, const double *f, double *b, int nrows, const int *ptr, const int *cell,
                const int *gidx, const double *coef, const double *g, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_active, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, mask, f, b);
    if (nrows)
        hipLaunchKernelGGL(k_rhs_rows, dim3((nrows + 255) / 256), dim3(256), 0, st, nrows, ptr, cell, gidx, coef, g, b);
}

void launch_zero_inactive(size_t n, const uint8_t *mask, double *u, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_inactive, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, mask, u);
}

void launch_gj_step(int n, int k, double *W, double *f, int *status, double tiny, hipStream_t st) {
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(1024), 0, st, n, k, W, f, status, tiny);
    const size_t cols = 2 * (size_t)n - (size_t)k;
    hipLaunchKernelGGL(k_gj_eliminate, dim3((unsigned)((cols + 255) / 256), (unsigned)((n + 3) / 4)), dim3(256), 0, st,
                       n, k, W, (const double *)f, (const int *)status);
}

void launch_fit(int m, const double *M, const double *phi, const double *w, const int *ncol, double *work,
                double *beta, int *status, hipStream_t st) {
    hipLaunchKernelGGL(k_fit, dim3((m + 63) / 64), dim3(64), 0, st, m, M, phi, w, ncol, work, beta, status);
}

template void launch_smooth_a<double>(const LevelArgs &, const double *, const double *, double *, const uint8_t *,
                                      bool, const PlgDev<double> &, hipStream_t, hipEvent_t, hipEvent_t);
template void launch_smooth_a<float>(const LevelArgs &, const float *, const float *, float *, const uint8_t *, bool,
                                     const PlgDev<float> &, hipStream_t, hipEvent_t, hipEvent_t);
template void launch_smooth_pair<double>(const LevelArgs &, const double *, const double *, double *, double *,
                                         const uint8_t *, bool, const PlgDev<double> &, const int *, int, const int *,
                                         int, hipStream_t, hipEvent_t, hipEvent_t);
template void launch_smooth_pair<float>(const LevelArgs &, const float *, const float *, float *, float *,
                                        const uint8_t *, bool, const PlgDev<float> &, const int *, int, const int *,
                                        int, hipStream_t, hipEvent_t, hipEvent_t);
template void launch_smooth_b<double>(const PlgDev<double> &, double *, hipStream_t);
template void launch_smooth_b<float>(const PlgDev<float> &, float *, hipStream_t);
template void launch_fill_zero<double>(size_t, double *, hipStream_t);
template void launch_fill_zero<float>(size_t, float *, hipStream_t);
template void launch_plg_residual<double>(int, const int *, const int *, const int *, const double *, const double *, const double *, double *, hipStream_t);
template void launch_plg_residual<float>(int, const int *, const int *, const int *, const float *, const float *, const float *, float *, hipStream_t);
template void launch_restrict<double>(const LevelArgs &, const LevelArgs &, const double *, const double *, const uint8_t *, const int *, const double *, const uint8_t *, double *, double *, int, const int *, const int *, const int *, bool, hipStream_t);
template void launch_restrict<float>(const LevelArgs &, const LevelArgs &, const float *, const float *, const uint8_t *, const int *, const float *, const uint8_t *, float *, float *, int, const int *, const int *, const int *, bool, hipStream_t);
template void launch_prolong<double>(const LevelArgs &, const LevelArgs &, const uint8_t *, const uint8_t *, const double *, double *, int, const int *, const int *, bool, hipStream_t);
template void launch_prolong<float>(const LevelArgs &, const LevelArgs &, const uint8_t *, const uint8_t *, const float *, float *, int, const int *, const int *, bool, hipStream_t);
template void launch_bottom<double, double>(int, const int *, const double *, const double *, double *, hipStream_t);
template void launch_bottom<float, float>(int, const int *, const double *, const float *, float *, hipStream_t);

}  // namespace mgc
