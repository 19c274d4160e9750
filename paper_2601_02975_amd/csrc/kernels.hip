// HIP kernels of the cut-cell V-cycle for CDNA4 (gfx950).
//
// Cell arrays are row-major with a halo of 2: cell (i, j) at
// (j + 2) * pitch + (i + 2), pitch = nx + 4.  The halo is never read as data:
// ghost values are synthesised from interior cells (Section 4.1).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "kernels_launch.hpp"

namespace mgc {

__constant__ double c_gw[2][2][4];     // [bc][depth-1][k] ghost weights on the cells k steps inward

hipError_t upload_ghost_table(const double gw[2][2][4]) {
    return hipMemcpyToSymbol(HIP_SYMBOL(c_gw), gw, sizeof(double) * 16);
}

__device__ __forceinline__ size_t pidx(const LevelArgs &L, int i, int j) {
    return (size_t)(j + 2) * L.pitch + (size_t)(i + 2);
}

// Ghost value at (qi, qj) outside the box, from the interior cells of the
// current iterate (homogeneous part; face data live in the right-hand side).
template <typename T>
__device__ T ghost_value(const T *__restrict__ u, const LevelArgs &L, int qi, int qj) {
    const bool ox = qi < 0 || qi >= L.nx, oy = qj < 0 || qj >= L.ny;
    if (ox && oy) {
        const int xside = qi < 0 ? 3 : 1, yside = qj < 0 ? 0 : 2;
        const int m = qi < 0 ? -qi : qi - L.nx + 1, k = qj < 0 ? -qj : qj - L.ny + 1;
        const double *gx = c_gw[L.bc[xside]][m - 1];
        const double *gy = c_gw[L.bc[yside]][k - 1];
        double s = 0.0;
        for (int p = 0; p < 4; ++p) {
            const int col = xside == 3 ? p : L.nx - 1 - p;
            double t = 0.0;
            for (int q = 0; q < 4; ++q) {
                const int row = yside == 0 ? q : L.ny - 1 - q;
                t += gy[q] * (double)u[pidx(L, col, row)];
            }
            s += gx[p] * t;
        }
        return (T)s;
    }
    int side, depth;
    if (qj < 0) { side = 0; depth = -qj; }
    else if (qj >= L.ny) { side = 2; depth = qj - L.ny + 1; }
    else if (qi < 0) { side = 3; depth = -qi; }
    else { side = 1; depth = qi - L.nx + 1; }
    const double *w = c_gw[L.bc[side]][depth - 1];
    double s = 0.0;
    for (int k = 0; k < 4; ++k) {
        int ci, cj;
        if (side == 0) { ci = qi; cj = k; }
        else if (side == 2) { ci = qi; cj = L.ny - 1 - k; }
        else if (side == 3) { ci = k; cj = qj; }
        else { ci = L.nx - 1 - k; cj = qj; }
        s += w[k] * (double)u[pidx(L, ci, cj)];
    }
    return (T)s;
}

template <typename T>
__device__ __forceinline__ T fetch(const T *__restrict__ u, const LevelArgs &L, int i, int j) {
    if (i >= 0 && i < L.nx && j >= 0 && j < L.ny) return u[pidx(L, i, j)];
    return ghost_value(u, L, i, j);
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

constexpr int TX = 64, TY = 32, HX = TX + 4, HY = TY + 4, NT = 256;

// Ghost value at (qi, qj) outside the box from a tile held in LDS; the tile
// origin (i0 - 2, j0 - 2) must contain the 4 interior cells next to the box
// edge in each direction the position lies beyond.
template <typename T>
__device__ __forceinline__ T ghost_lds(const T (*s)[HX], const LevelArgs &L, int i0, int j0, int qi, int qj) {
    auto at = [&](int i, int j) { return (double)s[j - j0 + 2][i - i0 + 2]; };
    const bool ox = qi < 0 || qi >= L.nx, oy = qj < 0 || qj >= L.ny;
    if (ox && oy) {
        const int xside = qi < 0 ? 3 : 1, yside = qj < 0 ? 0 : 2;
        const int m = qi < 0 ? -qi : qi - L.nx + 1, k = qj < 0 ? -qj : qj - L.ny + 1;
        const double *gx = c_gw[L.bc[xside]][m - 1];
        const double *gy = c_gw[L.bc[yside]][k - 1];
        double sum = 0.0;
        for (int p = 0; p < 4; ++p) {
            const int col = xside == 3 ? p : L.nx - 1 - p;
            double t = 0.0;
            for (int q = 0; q < 4; ++q) t += gy[q] * at(col, yside == 0 ? q : L.ny - 1 - q);
            sum += gx[p] * t;
        }
        return (T)sum;
    }
    int side, depth;
    if (qj < 0) { side = 0; depth = -qj; }
    else if (qj >= L.ny) { side = 2; depth = qj - L.ny + 1; }
    else if (qi < 0) { side = 3; depth = -qi; }
    else { side = 1; depth = qi - L.nx + 1; }
    const double *w = c_gw[L.bc[side]][depth - 1];
    double sum = 0.0;
    for (int k = 0; k < 4; ++k) {
        if (side == 0) sum += w[k] * at(qi, k);
        else if (side == 2) sum += w[k] * at(qi, L.ny - 1 - k);
        else if (side == 3) sum += w[k] * at(k, qj);
        else sum += w[k] * at(L.nx - 1 - k, qj);
    }
    return (T)sum;
}

// Loads the (TY+4) x (TX+4) tile with halo into LDS; halo positions outside
// the box are ghost values.  A block at the box edge first loads the interior
// cells, then fills the ghosts from LDS when the 4 cells inward from each
// edge it touches lie in the tile (always so when nx, ny are multiples of 4
// and at least 4 cells remain in the last tile), else from global memory.
template <typename T>
__device__ __forceinline__ void load_tile(T (*s)[HX], const T *__restrict__ u, const LevelArgs &L, int i0, int j0) {
    const bool edge = i0 < 2 || j0 < 2 || i0 + TX + 2 > L.nx || j0 + TY + 2 > L.ny;
    // all global loads of a thread are issued before any LDS store
    constexpr int NL = (HX * HY + NT - 1) / NT;
    T v[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int t = threadIdx.x + k * NT;
        const int ly = t / HX, lx = t - ly * HX;
        const int qi = i0 - 2 + lx, qj = j0 - 2 + ly;
        v[k] = (t < HX * HY && qi >= 0 && qi < L.nx && qj >= 0 && qj < L.ny) ? u[pidx(L, qi, qj)] : (T)0;
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int t = threadIdx.x + k * NT;
        if (t < HX * HY) s[t / HX][t % HX] = v[k];
    }
    if (!edge) return;
    // the tile holds cells [i0 - 2, i0 + TX + 2) x [j0 - 2, j0 + TY + 2);
    // the left and bottom edges (i0 = 0, j0 = 0) always have their 4 inward
    // cells in it, the right and top edges when nx - 4 >= i0 - 2 (ny - 4 >= j0 - 2)
    const bool lds_ok = (i0 + TX + 2 <= L.nx || L.nx - 4 >= i0 - 2) && (j0 + TY + 2 <= L.ny || L.ny - 4 >= j0 - 2);
    __syncthreads();
    for (int t = threadIdx.x; t < HX * HY; t += NT) {
        const int ly = t / HX, lx = t - ly * HX;
        const int qi = i0 - 2 + lx, qj = j0 - 2 + ly;
        const bool inside = qi >= 0 && qi < L.nx && qj >= 0 && qj < L.ny;
        if (!inside && qi >= -2 && qi < L.nx + 2 && qj >= -2 && qj < L.ny + 2)
            s[ly][lx] = lds_ok ? ghost_lds<T>(s, L, i0, j0, qi, qj) : ghost_value(u, L, qi, qj);
    }
}

// ---------------------------------------------------------------------------
// K1: weighted Jacobi on the SFV cells, eq. (5.5), D = -5(a+c)/(2h^2).
template <typename T, bool MIXED>
__global__ __launch_bounds__(NT) void k_jacobi(LevelArgs L, const T *__restrict__ uold, const T *__restrict__ b,
                                               T *__restrict__ unew, const uint8_t *__restrict__ mask) {
    __shared__ T s[HY][HX];
    constexpr int R = TY / (NT / TX);            // rows per thread
    const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int i = i0 + tx;
    // issue the per-cell loads before the tile barrier so that their latency
    // overlaps the tile load
    uint8_t mk[R];
    T bv[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int j = j0 + ty + k * (NT / TX);
        const bool in = i < L.nx && j < L.ny;
        const size_t id = pidx(L, in ? i : 0, in ? j : 0);
        mk[k] = in ? mask[id] : 0;
        bv[k] = b[id];
    }
    load_tile<T>(s, uold, L, i0, j0);
    __syncthreads();
    const T wod = (T)L.omega_over_d;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        if (mk[k] != 1) continue;
        const int r = ty + k * (NT / TX);
        const int lx = tx + 2, ly = r + 2;
        T au = apply_sfv<T, MIXED>(L, [&](int dx, int dy) { return s[ly + dy][lx + dx]; });
        unew[pidx(L, i, j0 + r)] = s[ly][lx] + wod * (bv[k] - au);
    }
}

// ---------------------------------------------------------------------------
// PLG rows: t = b2 - A21 u1 (eq. (5.6)), then u2 = A22^{-1} t via the
// segment / separator decomposition.
// Dense row-major blocks are applied one wavefront per row: the 64 lanes
// read consecutive columns (coalesced) and the partial sums are reduced
// across the wavefront.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

constexpr int PLG_ROWS = 32;     // rows per block in the PLG kernels (8 per wavefront)

// t = b2 - A21 u1 for all PLG rows (solve order): 32 lanes per row gather the
// row's SFV couplings in parallel.
template <typename T>
__global__ __launch_bounds__(256) void k_plg_gather(PlgDev<T> P, const T *__restrict__ b, const T *__restrict__ u,
                                                    T *__restrict__ t) {
    const int q = blockIdx.x * 8 + (threadIdx.x >> 5);
    const int lane = threadIdx.x & 31;
    if (q >= P.m) return;
    const int e0 = P.a21_ptr[q], e1 = P.a21_ptr[q + 1];
    T v = 0;
    for (int e = e0 + lane; e < e1; e += 32) v += P.a21_val[e] * u[P.a21_col[e]];
    for (int off = 16; off > 0; off >>= 1) v += __shfl_down(v, off, 32);
    if (lane == 0) t[q] = b[P.cell[q]] - v;
}

// P1: block (j, rb): rows [rb * PLG_ROWS, ...) of y_j = B_j^{-1} t_j
// (u2 = y_j if there are no separators)
template <typename T>
__global__ __launch_bounds__(256) void k_plg_seg(PlgDev<T> P, const T *__restrict__ tg, T *__restrict__ u) {
    extern __shared__ unsigned char smem_raw[];
    T *t = reinterpret_cast<T *>(smem_raw);
    const int j = blockIdx.x;
    const int s0 = P.seg_start[j], Lj = P.seg_start[j + 1] - s0;
    const int r0 = blockIdx.y * PLG_ROWS;
    if (r0 >= Lj) return;
    for (int r = threadIdx.x; r < Lj; r += blockDim.x) t[r] = tg[s0 + r];
    __syncthreads();
    const T *inv = P.inv + P.inv_off[j];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rw = r0 + wave * (PLG_ROWS / 4);
    T acc[PLG_ROWS / 4];
#pragma unroll
    for (int k = 0; k < PLG_ROWS / 4; ++k) acc[k] = 0;
    for (int c = lane; c < Lj; c += 64) {
        const T x = t[c];
#pragma unroll
        for (int k = 0; k < PLG_ROWS / 4; ++k)
            if (rw + k < Lj) acc[k] += inv[(size_t)(rw + k) * Lj + c] * x;
    }
#pragma unroll
    for (int k = 0; k < PLG_ROWS / 4; ++k) {
        const T a = wave_sum(acc[k]);
        if (lane == 0 && rw + k < Lj) {
            if (P.nsep == 0) u[P.cell[s0 + rw + k]] = a;
            else P.y[s0 + rw + k] = a;
        }
    }
}

// P2a: separator right-hand side r_S = t_S - A_SB y, 32 lanes per row
template <typename T>
__global__ __launch_bounds__(256) void k_plg_sep_rhs(PlgDev<T> P, const T *__restrict__ tg) {
    const int s = blockIdx.x * 8 + (threadIdx.x >> 5);
    const int lane = threadIdx.x & 31;
    if (s >= P.nsep) return;
    T v = 0;
    for (int e = P.sb_ptr[s] + lane; e < P.sb_ptr[s + 1]; e += 32) v += P.sb_val[e] * P.y[P.sb_col[e]];
    for (int off = 16; off > 0; off >>= 1) v += __shfl_down(v, off, 32);
    if (lane == 0) P.rs[s] = tg[P.sep_begin + s] - v;
}

// P2b: x_S = S'^{-1} r_S for the block's rows
template <typename T>
__global__ __launch_bounds__(256) void k_plg_sep(PlgDev<T> P, T *__restrict__ u) {
    extern __shared__ unsigned char smem_raw[];
    T *rs = reinterpret_cast<T *>(smem_raw);
    const int ns = P.nsep;
    for (int s = threadIdx.x; s < ns; s += blockDim.x) rs[s] = P.rs[s];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r0 = blockIdx.x * PLG_ROWS + wave * (PLG_ROWS / 4);
    T acc[PLG_ROWS / 4];
#pragma unroll
    for (int k = 0; k < PLG_ROWS / 4; ++k) acc[k] = 0;
    for (int c = lane; c < ns; c += 64) {
        const T x = rs[c];
#pragma unroll
        for (int k = 0; k < PLG_ROWS / 4; ++k)
            if (r0 + k < ns) acc[k] += P.sinv[(size_t)(r0 + k) * ns + c] * x;
    }
#pragma unroll
    for (int k = 0; k < PLG_ROWS / 4; ++k) {
        const T a = wave_sum(acc[k]);
        if (lane == 0 && r0 + k < ns) {
            P.xs[r0 + k] = a;
            u[P.cell[P.sep_begin + r0 + k]] = a;
        }
    }
}

// P3: x_j = y_j - F_j x_S (F_j row-major, L_j x k_j)
template <typename T>
__global__ __launch_bounds__(256) void k_plg_fix(PlgDev<T> P, T *__restrict__ u) {
    const int j = blockIdx.x;
    const int s0 = P.seg_start[j], Lj = P.seg_start[j + 1] - s0;
    const int k0 = P.fcols_ptr[j], k = P.fcols_ptr[j + 1] - k0;
    const T *F = P.F + P.f_off[j];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r0 = blockIdx.y * PLG_ROWS;
    for (int r = r0 + wave; r < min(r0 + PLG_ROWS, Lj); r += 4) {
        T acc = 0;
        for (int kk = lane; kk < k; kk += 64) acc += F[(size_t)r * k + kk] * P.xs[P.fcols[k0 + kk]];
        acc = wave_sum(acc);
        if (lane == 0) u[P.cell[s0 + r]] = P.y[s0 + r] - acc;
    }
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

// K2: residual of the fine level fused with the restriction of eq. (5.8):
// one thread per coarse cell, children summed with weight 1/4; zero the
// coarse initial guess.
template <typename T, bool MIXED>
__global__ __launch_bounds__(NT) void k_restrict(LevelArgs L, LevelArgs C, const T *__restrict__ u,
                                                 const T *__restrict__ b, const uint8_t *__restrict__ mask,
                                                 const int *__restrict__ plgidx, const T *__restrict__ rplg,
                                                 const uint8_t *__restrict__ cmask, T *__restrict__ bc,
                                                 T *__restrict__ uc) {
    __shared__ T s[HY][HX];
    const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY;
    constexpr int NC = (TX / 2) * (TY / 2) / NT;      // coarse cells per thread
    uint8_t ck[NC], fk[NC][4];
    T fb[NC][4];
#pragma unroll
    for (int n = 0; n < NC; ++n) {
        const int t = threadIdx.x + n * NT;
        const int ci = blockIdx.x * (TX / 2) + t % (TX / 2), cj = blockIdx.y * (TY / 2) + t / (TX / 2);
        const bool cin = ci < C.nx && cj < C.ny;
        ck[n] = cin ? cmask[pidx(C, ci, cj)] : 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int fi = 2 * ci + (q & 1), fj = 2 * cj + (q >> 1);
            const bool fin = cin && fi < L.nx && fj < L.ny;
            const size_t id = pidx(L, fin ? fi : 0, fin ? fj : 0);
            fk[n][q] = fin ? mask[id] : 0;
            fb[n][q] = b[id];
        }
    }
    load_tile<T>(s, u, L, i0, j0);
    __syncthreads();
#pragma unroll
    for (int n = 0; n < NC; ++n) {
        const int t = threadIdx.x + n * NT;
        const int ci = blockIdx.x * (TX / 2) + t % (TX / 2), cj = blockIdx.y * (TY / 2) + t / (TX / 2);
        if (ci >= C.nx || cj >= C.ny) continue;
        const size_t cid = pidx(C, ci, cj);
        uc[cid] = 0;
        T sum = 0;
        if (ck[n]) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int fi = 2 * ci + (q & 1), fj = 2 * cj + (q >> 1);
                if (fk[n][q] == 1) {
                    const int lx = fi - i0 + 2, ly = fj - j0 + 2;
                    sum += fb[n][q] - apply_sfv<T, MIXED>(L, [&](int dx, int dy) { return s[ly + dy][lx + dx]; });
                } else if (fk[n][q] == 2) {
                    sum += rplg[plgidx[pidx(L, fi, fj)]];
                }
            }
        }
        bc[cid] = (T)0.25 * sum;
    }
}

// fine cells whose coarse parent was merged away: add to the absorbing cell
template <typename T, bool MIXED>
__global__ void k_restrict_ex(LevelArgs L, LevelArgs C, int nt, const int *__restrict__ ptr,
                              const int *__restrict__ target, const int *__restrict__ child,
                              const T *__restrict__ u, const T *__restrict__ b, const uint8_t *__restrict__ mask,
                              const int *__restrict__ plgidx, const T *__restrict__ rplg, T *__restrict__ bc) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    T sum = 0;
    for (int e = ptr[t]; e < ptr[t + 1]; ++e) {
        const int id = child[e];
        const int i = id % L.pitch - 2, j = id / L.pitch - 2;
        if (mask[id] == 1) {
            sum += b[id] - apply_sfv<T, MIXED>(L, [&](int dx, int dy) { return fetch(u, L, i + dx, j + dy); });
        } else if (mask[id] == 2) {
            sum += rplg[plgidx[id]];
        }
    }
    bc[target[t]] += (T)0.25 * sum;
}

// K3: piecewise-constant interpolation and correction, eq. (5.9)
template <typename T>
__global__ void k_prolong(LevelArgs L, LevelArgs C, const uint8_t *__restrict__ mask,
                          const uint8_t *__restrict__ cmask, const T *__restrict__ ec, T *__restrict__ u) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= L.nx) return;
    const size_t id = pidx(L, i, j);
    const size_t cid = pidx(C, i >> 1, j >> 1);
    if (mask[id] && cmask[cid]) u[id] += ec[cid];
}

template <typename T>
__global__ void k_prolong_ex(int n, const int *__restrict__ fine, const int *__restrict__ coarse,
                             const T *__restrict__ ec, T *__restrict__ u) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) u[fine[k]] += ec[coarse[k]];
}

// ---------------------------------------------------------------------------
// K6: bottom solve x = A_c^{-1} b (FP64 dense inverse, row-major): one
// wavefront per row, 16 wavefronts per block, the right-hand side staged in
// LDS by every block.
constexpr int BOT_WAVES = 16;
template <typename TI, typename TO>
__global__ __launch_bounds__(64 * BOT_WAVES) void k_bottom(int n, const int *__restrict__ cells,
                                                          const double *__restrict__ ainv, const TI *__restrict__ b,
                                                          TO *__restrict__ x) {
    extern __shared__ unsigned char smem_raw[];
    double *bs = reinterpret_cast<double *>(smem_raw);
    for (int k = threadIdx.x; k < n; k += blockDim.x) bs[k] = (double)b[cells[k]];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = blockIdx.x * BOT_WAVES + wave;
    if (row >= n) return;
    const double *a = ainv + (size_t)row * n;
    double acc = 0.0;
    for (int c = lane; c < n; c += 64) acc += a[c] * bs[c];
    acc = wave_sum(acc);
    if (lane == 0) x[cells[row]] = (TO)acc;
}

// ---------------------------------------------------------------------------
// K7: residual max-norm over active cells (SFV by the stencil, PLG from
// rplg); optionally writes r as FP32 (mixed-precision defect correction).
template <bool MIXED, bool WRITE32>
__global__ __launch_bounds__(NT) void k_residual_norm(LevelArgs L, const double *__restrict__ u,
                                                      const double *__restrict__ b, const uint8_t *__restrict__ mask,
                                                      const int *__restrict__ plgidx, const double *__restrict__ rplg,
                                                      float *__restrict__ r32, double *__restrict__ r64,
                                                      double *__restrict__ partial) {
    __shared__ double s[HY][HX];
    __shared__ double red[NT];
    constexpr int R = TY / (NT / TX);
    const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int i = i0 + tx;
    uint8_t mk[R];
    double bv[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int j = j0 + ty + k * (NT / TX);
        const bool in = i < L.nx && j < L.ny;
        const size_t id = pidx(L, in ? i : 0, in ? j : 0);
        mk[k] = in ? mask[id] : 0;
        bv[k] = b[id];
    }
    load_tile<double>(s, u, L, i0, j0);
    __syncthreads();
    double mx = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int rr = ty + k * (NT / TX);
        const int j = j0 + rr;
        if (i >= L.nx || j >= L.ny) continue;
        const size_t id = pidx(L, i, j);
        double r = 0.0;
        if (mk[k] == 1) {
            const int lx = tx + 2, ly = rr + 2;
            r = bv[k] - apply_sfv<double, MIXED>(L, [&](int dx, int dy) { return s[ly + dy][lx + dx]; });
        } else if (mk[k] == 2) {
            r = rplg[plgidx[id]];
        }
        if (WRITE32) r32[id] = (float)r;
        if (r64) r64[id] = r;
        mx = fmax(mx, fabs(r));
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int off = NT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
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

// K8: b = f - N g (eq. (4.19)) on the finest level
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

// K9: u64 += e32 over active cells; zero inactive cells
__global__ void k_add_correction(size_t n, const uint8_t *__restrict__ mask, const float *__restrict__ e,
                                 double *__restrict__ u) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n && mask[k]) u[k] += (double)e[k];
}

__global__ void k_fill_zero_f32(size_t n, float *__restrict__ u) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) u[k] = 0.0f;
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
void launch_jacobi(const LevelArgs &L, const T *uold, const T *b, T *unew, const uint8_t *mask, hipStream_t st) {
    if (L.mixed) hipLaunchKernelGGL((k_jacobi<T, true>), tile_grid(L), dim3(NT), 0, st, L, uold, b, unew, mask);
    else hipLaunchKernelGGL((k_jacobi<T, false>), tile_grid(L), dim3(NT), 0, st, L, uold, b, unew, mask);
}

template <typename T>
void launch_plg_solve(const PlgDev<T> &P, const T *b, T *u, hipStream_t st) {
    if (P.m == 0) return;
    const unsigned rb = (P.max_seg + PLG_ROWS - 1) / PLG_ROWS;
    hipLaunchKernelGGL((k_plg_gather<T>), dim3((P.m + 7) / 8), dim3(256), 0, st, P, b, u, P.t);
    if (P.nseg) hipLaunchKernelGGL((k_plg_seg<T>), dim3(P.nseg, rb), dim3(256), sizeof(T) * P.max_seg, st, P, P.t, u);
    if (P.nsep) {
        hipLaunchKernelGGL((k_plg_sep_rhs<T>), dim3((P.nsep + 7) / 8), dim3(256), 0, st, P, P.t);
        hipLaunchKernelGGL((k_plg_sep<T>), dim3((P.nsep + PLG_ROWS - 1) / PLG_ROWS), dim3(256), sizeof(T) * P.nsep, st,
                           P, u);
        if (P.nseg) hipLaunchKernelGGL((k_plg_fix<T>), dim3(P.nseg, rb), dim3(256), 0, st, P, u);
    }
}

template <typename T>
void launch_plg_residual(int m, const int *cell, const int *ptr, const int *col, const T *val, const T *b,
                         const T *u, T *r, hipStream_t st) {
    if (m == 0) return;
    hipLaunchKernelGGL((k_plg_residual<T>), dim3((m + 255) / 256), dim3(256), 0, st, m, cell, ptr, col, val, b, u, r);
}

template <typename T>
void launch_restrict(const LevelArgs &L, const LevelArgs &C, const T *u, const T *b, const uint8_t *mask,
                     const int *plgidx, const T *rplg, const uint8_t *cmask, T *bc, T *uc, int nt, const int *ex_ptr,
                     const int *ex_target, const int *ex_child, hipStream_t st) {
    dim3 grid((C.nx + TX / 2 - 1) / (TX / 2), (C.ny + TY / 2 - 1) / (TY / 2));
    if (L.mixed)
        hipLaunchKernelGGL((k_restrict<T, true>), grid, dim3(NT), 0, st, L, C, u, b, mask, plgidx, rplg, cmask, bc, uc);
    else
        hipLaunchKernelGGL((k_restrict<T, false>), grid, dim3(NT), 0, st, L, C, u, b, mask, plgidx, rplg, cmask, bc, uc);
    if (nt) {
        if (L.mixed)
            hipLaunchKernelGGL((k_restrict_ex<T, true>), dim3((nt + 63) / 64), dim3(64), 0, st, L, C, nt, ex_ptr,
                               ex_target, ex_child, u, b, mask, plgidx, rplg, bc);
        else
            hipLaunchKernelGGL((k_restrict_ex<T, false>), dim3((nt + 63) / 64), dim3(64), 0, st, L, C, nt, ex_ptr,
                               ex_target, ex_child, u, b, mask, plgidx, rplg, bc);
    }
}

template <typename T>
void launch_prolong(const LevelArgs &L, const LevelArgs &C, const uint8_t *mask, const uint8_t *cmask, const T *ec,
                    T *u, int nex, const int *ex_fine, const int *ex_coarse, hipStream_t st) {
    hipLaunchKernelGGL((k_prolong<T>), dim3((L.nx + 255) / 256, L.ny), dim3(256), 0, st, L, C, mask, cmask, ec, u);
    if (nex)
        hipLaunchKernelGGL((k_prolong_ex<T>), dim3((nex + 255) / 256), dim3(256), 0, st, nex, ex_fine, ex_coarse, ec, u);
}

template <typename TI, typename TO>
void launch_bottom(int n, const int *cells, const double *ainv, const TI *b, TO *x, hipStream_t st) {
    hipLaunchKernelGGL((k_bottom<TI, TO>), dim3((n + BOT_WAVES - 1) / BOT_WAVES), dim3(64 * BOT_WAVES),
                       sizeof(double) * n, st, n, cells, ainv, b, x);
}

int launch_residual_norm(const LevelArgs &L, const double *u, const double *b, const uint8_t *mask, const int *plgidx,
                         const double *rplg, float *r32, double *r64, double *partial, hipStream_t st) {
    dim3 g = tile_grid(L);
    if (r32) {
        if (L.mixed) hipLaunchKernelGGL((k_residual_norm<true, true>), g, dim3(NT), 0, st, L, u, b, mask, plgidx, rplg, r32, r64, partial);
        else hipLaunchKernelGGL((k_residual_norm<false, true>), g, dim3(NT), 0, st, L, u, b, mask, plgidx, rplg, r32, r64, partial);
    } else {
        if (L.mixed) hipLaunchKernelGGL((k_residual_norm<true, false>), g, dim3(NT), 0, st, L, u, b, mask, plgidx, rplg, r32, r64, partial);
        else hipLaunchKernelGGL((k_residual_norm<false, false>), g, dim3(NT), 0, st, L, u, b, mask, plgidx, rplg, r32, r64, partial);
    }
    return (int)(g.x * g.y);
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

void launch_add_correction(size_t n, const uint8_t *mask, const float *e, double *u, hipStream_t st) {
    hipLaunchKernelGGL(k_add_correction, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, mask, e, u);
}

void launch_fill_zero(size_t n, float *u, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_zero_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, u);
}

void launch_zero_inactive(size_t n, const uint8_t *mask, double *u, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_inactive, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, mask, u);
}

void launch_fit(int m, const double *M, const double *phi, const double *w, const int *ncol, double *work,
                double *beta, int *status, hipStream_t st) {
    hipLaunchKernelGGL(k_fit, dim3((m + 63) / 64), dim3(64), 0, st, m, M, phi, w, ncol, work, beta, status);
}

template void launch_jacobi<double>(const LevelArgs &, const double *, const double *, double *, const uint8_t *, hipStream_t);
template void launch_jacobi<float>(const LevelArgs &, const float *, const float *, float *, const uint8_t *, hipStream_t);
template void launch_plg_solve<double>(const PlgDev<double> &, const double *, double *, hipStream_t);
template void launch_plg_solve<float>(const PlgDev<float> &, const float *, float *, hipStream_t);
template void launch_plg_residual<double>(int, const int *, const int *, const int *, const double *, const double *, const double *, double *, hipStream_t);
template void launch_plg_residual<float>(int, const int *, const int *, const int *, const float *, const float *, const float *, float *, hipStream_t);
template void launch_restrict<double>(const LevelArgs &, const LevelArgs &, const double *, const double *, const uint8_t *, const int *, const double *, const uint8_t *, double *, double *, int, const int *, const int *, const int *, hipStream_t);
template void launch_restrict<float>(const LevelArgs &, const LevelArgs &, const float *, const float *, const uint8_t *, const int *, const float *, const uint8_t *, float *, float *, int, const int *, const int *, const int *, hipStream_t);
template void launch_prolong<double>(const LevelArgs &, const LevelArgs &, const uint8_t *, const uint8_t *, const double *, double *, int, const int *, const int *, hipStream_t);
template void launch_prolong<float>(const LevelArgs &, const LevelArgs &, const uint8_t *, const uint8_t *, const float *, float *, int, const int *, const int *, hipStream_t);
template void launch_bottom<double, double>(int, const int *, const double *, const double *, double *, hipStream_t);
template void launch_bottom<float, float>(int, const int *, const double *, const float *, float *, hipStream_t);

}  // namespace mgc
