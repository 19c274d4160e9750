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

constexpr int TX = 64, TY = 16, HX = TX + 4, HY = TY + 4, NT = 256;

// Loads the (TY+4) x (TX+4) tile with halo into LDS; halo positions outside
// the box are filled with ghost values (only blocks touching the box edge).
template <typename T>
__device__ __forceinline__ void load_tile(T (*s)[HX], const T *__restrict__ u, const LevelArgs &L, int i0, int j0) {
    const bool edge = i0 < 2 || j0 < 2 || i0 + TX + 2 > L.nx || j0 + TY + 2 > L.ny;
    for (int t = threadIdx.x; t < HX * HY; t += NT) {
        const int ly = t / HX, lx = t - ly * HX;
        const int qi = i0 - 2 + lx, qj = j0 - 2 + ly;
        T v = 0;
        if (qi >= 0 && qi < L.nx && qj >= 0 && qj < L.ny) v = u[pidx(L, qi, qj)];
        else if (edge && qi >= -2 && qi < L.nx + 2 && qj >= -2 && qj < L.ny + 2) v = ghost_value(u, L, qi, qj);
        s[ly][lx] = v;
    }
}

// ---------------------------------------------------------------------------
// K1: weighted Jacobi on the SFV cells, eq. (5.5), D = -5(a+c)/(2h^2).
template <typename T, bool MIXED>
__global__ __launch_bounds__(NT) void k_jacobi(LevelArgs L, const T *__restrict__ uold, const T *__restrict__ b,
                                               T *__restrict__ unew, const uint8_t *__restrict__ mask) {
    __shared__ T s[HY][HX];
    const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY;
    load_tile<T>(s, uold, L, i0, j0);
    __syncthreads();
    const int tx = threadIdx.x % TX;
    const T wod = (T)L.omega_over_d;
    for (int r = threadIdx.x / TX; r < TY; r += NT / TX) {
        const int i = i0 + tx, j = j0 + r;
        if (i >= L.nx || j >= L.ny) continue;
        const size_t id = pidx(L, i, j);
        if (mask[id] != 1) continue;
        const int lx = tx + 2, ly = r + 2;
        T au = apply_sfv<T, MIXED>(L, [&](int dx, int dy) { return s[ly + dy][lx + dx]; });
        unew[id] = s[ly][lx] + wod * (b[id] - au);
    }
}

// ---------------------------------------------------------------------------
// PLG rows: t = b2 - A21 u1 (eq. (5.6)), then u2 = A22^{-1} t via the
// segment / separator decomposition.
// P1: one block per segment: t_j, y_j = B_j^{-1} t_j (u2 = y_j if no separators)
template <typename T>
__global__ __launch_bounds__(256) void k_plg_seg(PlgDev<T> P, const T *__restrict__ b, T *__restrict__ u) {
    extern __shared__ unsigned char smem_raw[];
    T *t = reinterpret_cast<T *>(smem_raw);
    const int j = blockIdx.x;
    const int s0 = P.seg_start[j], Lj = P.seg_start[j + 1] - s0;
    for (int r = threadIdx.x; r < Lj; r += blockDim.x) {
        const int q = s0 + r;
        T v = b[P.cell[q]];
        for (int e = P.a21_ptr[q]; e < P.a21_ptr[q + 1]; ++e) v -= P.a21_val[e] * u[P.a21_col[e]];
        t[r] = v;
    }
    __syncthreads();
    const T *inv = P.inv + P.inv_off[j];
    for (int r = threadIdx.x; r < Lj; r += blockDim.x) {
        T acc = 0;
        for (int c = 0; c < Lj; ++c) acc += inv[(size_t)c * Lj + r] * t[c];
        if (P.nsep == 0) u[P.cell[s0 + r]] = acc;
        else P.y[s0 + r] = acc;
    }
}

// P2: separators: r_S = t_S - A_SB y, x_S = S'^{-1} r_S (each block recomputes r_S)
template <typename T>
__global__ __launch_bounds__(256) void k_plg_sep(PlgDev<T> P, const T *__restrict__ b, T *__restrict__ u) {
    extern __shared__ unsigned char smem_raw[];
    T *rs = reinterpret_cast<T *>(smem_raw);
    const int ns = P.nsep;
    for (int s = threadIdx.x; s < ns; s += blockDim.x) {
        const int q = P.sep_begin + s;
        T v = b[P.cell[q]];
        for (int e = P.a21_ptr[q]; e < P.a21_ptr[q + 1]; ++e) v -= P.a21_val[e] * u[P.a21_col[e]];
        for (int e = P.sb_ptr[s]; e < P.sb_ptr[s + 1]; ++e) v -= P.sb_val[e] * P.y[P.sb_col[e]];
        rs[s] = v;
    }
    __syncthreads();
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row < ns) {
        T acc = 0;
        for (int c = 0; c < ns; ++c) acc += P.sinv[(size_t)c * ns + row] * rs[c];
        P.xs[row] = acc;
        u[P.cell[P.sep_begin + row]] = acc;
    }
}

// P3: x_j = y_j - F_j x_S
template <typename T>
__global__ __launch_bounds__(256) void k_plg_fix(PlgDev<T> P, T *__restrict__ u) {
    const int j = blockIdx.x;
    const int s0 = P.seg_start[j], Lj = P.seg_start[j + 1] - s0;
    const int k0 = P.fcols_ptr[j], k = P.fcols_ptr[j + 1] - k0;
    const T *F = P.F + P.f_off[j];
    for (int r = threadIdx.x; r < Lj; r += blockDim.x) {
        T acc = P.y[s0 + r];
        for (int kk = 0; kk < k; ++kk) acc -= F[(size_t)kk * Lj + r] * P.xs[P.fcols[k0 + kk]];
        u[P.cell[s0 + r]] = acc;
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
    load_tile<T>(s, u, L, i0, j0);
    __syncthreads();
    const int ci = blockIdx.x * (TX / 2) + threadIdx.x % (TX / 2);
    const int cj = blockIdx.y * (TY / 2) + threadIdx.x / (TX / 2);
    if (ci >= C.nx || cj >= C.ny) return;
    const size_t cid = pidx(C, ci, cj);
    uc[cid] = 0;
    if (!cmask[cid]) {
        bc[cid] = 0;
        return;
    }
    T sum = 0;
#pragma unroll
    for (int dj = 0; dj < 2; ++dj)
#pragma unroll
        for (int di = 0; di < 2; ++di) {
            const int i = 2 * ci + di, j = 2 * cj + dj;
            if (i >= L.nx || j >= L.ny) continue;
            const size_t id = pidx(L, i, j);
            const uint8_t k = mask[id];
            if (k == 1) {
                const int lx = i - i0 + 2, ly = j - j0 + 2;
                sum += b[id] - apply_sfv<T, MIXED>(L, [&](int dx, int dy) { return s[ly + dy][lx + dx]; });
            } else if (k == 2) {
                sum += rplg[plgidx[id]];
            }
        }
    bc[cid] = (T)0.25 * sum;
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
// K6: bottom solve x = A_c^{-1} b (FP64 dense inverse, row-major); one
// wavefront per row, the right-hand side staged in LDS.
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_bottom(int n, const int *__restrict__ cells, const double *__restrict__ ainv,
                                                const TI *__restrict__ b, TO *__restrict__ x) {
    extern __shared__ unsigned char smem_raw[];
    double *bs = reinterpret_cast<double *>(smem_raw);
    for (int k = threadIdx.x; k < n; k += blockDim.x) bs[k] = (double)b[cells[k]];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rows_per_block = 16;
    for (int rr = wave; rr < rows_per_block; rr += 4) {
        const int row = blockIdx.x * rows_per_block + rr;
        if (row >= n) break;
        const double *a = ainv + (size_t)row * n;
        double acc = 0.0;
        for (int c = lane; c < n; c += 64) acc += a[c] * bs[c];
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        if (lane == 0) x[cells[row]] = (TO)acc;
    }
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
    const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY;
    load_tile<double>(s, u, L, i0, j0);
    __syncthreads();
    const int tx = threadIdx.x % TX;
    double mx = 0.0;
    for (int rr = threadIdx.x / TX; rr < TY; rr += NT / TX) {
        const int i = i0 + tx, j = j0 + rr;
        if (i >= L.nx || j >= L.ny) continue;
        const size_t id = pidx(L, i, j);
        const uint8_t k = mask[id];
        double r = 0.0;
        if (k == 1) {
            const int lx = tx + 2, ly = rr + 2;
            r = b[id] - apply_sfv<double, MIXED>(L, [&](int dx, int dy) { return s[ly + dy][lx + dx]; });
        } else if (k == 2) {
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
    if (P.nseg) hipLaunchKernelGGL((k_plg_seg<T>), dim3(P.nseg), dim3(256), sizeof(T) * P.max_seg, st, P, b, u);
    if (P.nsep) {
        hipLaunchKernelGGL((k_plg_sep<T>), dim3((P.nsep + 255) / 256), dim3(256), sizeof(T) * P.nsep, st, P, b, u);
        if (P.nseg) hipLaunchKernelGGL((k_plg_fix<T>), dim3(P.nseg), dim3(256), 0, st, P, u);
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
    hipLaunchKernelGGL((k_bottom<TI, TO>), dim3((n + 15) / 16), dim3(256), sizeof(double) * n, st, n, cells, ainv, b, x);
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
