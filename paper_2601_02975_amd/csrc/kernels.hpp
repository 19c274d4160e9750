// Device-side level description and kernel launchers (CDNA4 / gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mgc {

constexpr uint8_t FULL_ALL_SFV = 1, FULL_NO_SFV = 2, FULL_DEAD = 4;

// rows of the SFV tiles (64 cells wide) of a split launch A, by word size
constexpr int split_tile_rows(int word) { return word == 4 ? 32 : 16; }

// Launch-time parameters of one level (passed by value).
struct LevelArgs {
    int nx, ny, pitch;          // pitch = nx + 4, origin at (2, 2)
    double h;
    double cxx, cxy, cyy;       // a/h^2, b/h^2, c/h^2
    double omega_over_d;        // omega / D, D = -5(a+c)/(2h^2)
    // ghost weights on the 4 interior cells (homogeneous part; boundary data
    // enter through the right-hand side), device array gw[(side * 2 + depth - 1) * 4 + k],
    // sides bottom, right, top, left, k = steps inward
    const double *gw;
    // per block of 64 x 8 cells (row-major, full_bx x full_by blocks), flags:
    // FULL_ALL_SFV, every cell is an SFV cell (tiles made of such blocks need
    // not read the class bytes); FULL_NO_SFV, no cell is (the smoother's
    // tiles have nothing to update); FULL_DEAD, no cell is active, nor any of
    // the 32 x 4 cells of the next coarser level under the block (the
    // residual and restriction tiles would only write zeros that are already
    // there)
    const uint8_t *full;
    int full_bx, full_by;
    // tiles of 64 x 32 cells (row-major tile numbers) that hold an active
    // cell or lie over one of the next coarser level, in order; the
    // residual and restriction launch only these on the hierarchy's own
    // buffers (null: every tile is such a tile)
    const int *live;
    int nlive;
    int mixed;                  // b != 0
    // launch shape of the smoother's launch A on this level (chosen at setup
    // from the grid size, or forced by the options): split_a = 1 runs the
    // SFV tiles and the PLG groups as two kernels; small32 / small64 = 1
    // selects 8-row tiles for the fused kernel in FP32 / FP64
    int split_a, small32, small64;
    int colouring;              // 1: the multicolour variant of the SFV half of the smoother
    int periodic;               // bit 0: left/right sides periodic, bit 1: bottom/top sides periodic
};

// Launch A PLG block: rows [r0, r1) of group g (rows [gs, gs + n) in solve
// order, SFV couplings H = hcell[h0, h0 + nh)); segment groups also carry
// their inverse and their entries of A_SB [ce0, ce1).
struct alignas(16) PlgBlkA {
    int g, r0, r1, gs;
    int n, h0, nh, ce0;
    int ce1, pad0;
    long long inv_off;
};

// Launch B block: kind 0, rows [r0, r1) of segment j (rows [s0, s0 + Lj),
// k_j separator columns); kind 1, separator rows [r0, r1).
struct alignas(16) PlgBlkB {
    int kind, j, r0, r1;
    int kj, s0, Lj, pad0;
    long long sj_off, ft_off;
};

// PLG block solve data of one level (device pointers).  Rows are numbered
// in solve order: the segments (consecutive runs), then the separators.
// Row-wise sparse data have a fixed width of ELL_W entries (zero padding).
template <typename T>
struct PlgDev {
    int m = 0, nseg = 0, nsep = 0, sep_begin = 0;
    const int *cell = nullptr;          // [m] padded cell index
    // gather groups (launch A)
    const int *grp_start = nullptr;     // [ngroup + 1]
    const int *hptr = nullptr, *hcell = nullptr;   // SFV cells coupled to each group
    const int *a21_loc = nullptr;       // [m * ELL_W] index into the group's H
    const T *a21_val = nullptr;
    int nblk1 = 0;
    const PlgBlkA *blk1 = nullptr;
    // segments
    const int *seg_start = nullptr;     // [nseg + 1]
    const long long *inv_off = nullptr; // row-major segment inverses
    const T *inv = nullptr;
    const int *ce_ptr = nullptr, *ce_row = nullptr, *ce_slot = nullptr;   // A_SB entries on each segment's rows
    const T *ce_val = nullptr;
    // separators (launch B)
    int nblk2 = 0;
    const PlgBlkB *blk2 = nullptr;
    const long long *ft_off = nullptr;  // F_j^T = (B_j^{-1} A_{j,S})^T, row-major k_j x L_j
    const T *FT = nullptr;
    const int *fcols_ptr = nullptr;     // k_j = fcols_ptr[j + 1] - fcols_ptr[j]
    const int *fcols = nullptr;         // separator index of each of those columns
    int nblk2_seg = 0;                  // launch B blocks of segment slices (they come first)
    int split_b = 0;                    // launch B as two kernels (separator rows, then segment slices)
    const long long *sj_off = nullptr;  // rows of S'^{-1} at segment j's separator columns, k_j x nsep
    const T *SJ = nullptr;
    const T *sinv = nullptr;            // row-major nsep x nsep
    T *t = nullptr;                     // [m] separator right-hand sides b2 - A21 u1
    T *y = nullptr;                     // [m] segment solutions B^{-1} t
    T *contrib = nullptr;               // [nsep * ELL_W] entries of A_SB times y
};

constexpr int ELL_W = 16;               // width of the row-wise sparse data

// Limits of the LDS staging (checked at setup).
constexpr int PLG_HMAX = 1536;          // SFV cells coupled to one group
constexpr int PLG_LMAX = 768;           // rows of one group
constexpr int PLG_KMAX = 256;           // separator columns of one segment
constexpr int PLG_SMAX = 4096;          // separator rows of one level
constexpr int PLG_SLICE = 32;           // segment rows per block
constexpr int PLG_B_ROWS = 32;          // segment rows per block of launch B (one per thread)
constexpr int PLG_SEP_ROWS = 16;        // separator rows per block of launch B

}  // namespace mgc
