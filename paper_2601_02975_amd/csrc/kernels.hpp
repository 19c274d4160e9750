// Device-side level description and kernel launchers (CDNA4 / gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mgc {

// Ghost weights on the 4 interior cells (homogeneous part; boundary data
// enter through the right-hand side).  gw[bc][depth-1][k], bc 0 Dirichlet,
// 1 Neumann; k = steps inward.
struct GhostTable {
    double gw[2][2][4];
    double face[2][2];          // face-datum weights (for reference)
    double ext[2][4];           // cubic extrapolation along a face
};

// Launch-time parameters of one level (passed by value).
struct LevelArgs {
    int nx, ny, pitch;          // pitch = nx + 4, origin at (2, 2)
    double h;
    double cxx, cxy, cyy;       // a/h^2, b/h^2, c/h^2
    double omega_over_d;        // omega / D, D = -5(a+c)/(2h^2)
    int bc[4];                  // box sides: bottom, right, top, left (0 D, 1 N)
    int mixed;                  // b != 0
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
    const int4 *blk1 = nullptr;         // (group, r0, r1, -)
    // segments
    const int *seg_start = nullptr;     // [nseg + 1]
    const long long *inv_off = nullptr; // row-major segment inverses
    const T *inv = nullptr;
    const int *ce_ptr = nullptr, *ce_row = nullptr, *ce_slot = nullptr;   // A_SB entries on each segment's rows
    const T *ce_val = nullptr;
    // separators (launch B)
    int nblk2 = 0;
    const int4 *blk2 = nullptr;         // (0 segment slice | 1 separator rows, j, r0, r1)
    const long long *ft_off = nullptr;  // F_j^T = (B_j^{-1} A_{j,S})^T, row-major k_j x L_j
    const T *FT = nullptr;
    const int *fcols_ptr = nullptr;     // k_j = fcols_ptr[j + 1] - fcols_ptr[j]
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
constexpr int PLG_LMAX = 320;           // rows of one group (segments reach 1.25x the nominal 256)
constexpr int PLG_KMAX = 256;           // separator columns of one segment
constexpr int PLG_SMAX = 4096;          // separator rows of one level
constexpr int PLG_SLICE = 32;           // segment rows per block
constexpr int PLG_SEP_ROWS = 32;        // separator rows per block of launch B

}  // namespace mgc
