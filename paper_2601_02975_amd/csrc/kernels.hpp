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

// PLG block solve data of one level (device pointers)
template <typename T>
struct PlgDev {
    int m = 0, nseg = 0, nsep = 0, sep_begin = 0;
    const int *cell = nullptr;          // [m] padded cell index, solve order
    const int *a21_ptr = nullptr;       // [m+1] SFV couplings of each PLG row (solve order)
    const int *a21_col = nullptr;       // padded cell index
    const T *a21_val = nullptr;
    const int *seg_start = nullptr;     // [nseg+1]
    const long long *inv_off = nullptr; // [nseg]
    const T *inv = nullptr;             // row-major segment inverses
    const long long *f_off = nullptr;
    const T *F = nullptr;
    const int *fcols_ptr = nullptr, *fcols = nullptr;
    const T *sinv = nullptr;            // row-major
    const int *sb_ptr = nullptr, *sb_col = nullptr;   // separator rows -> segment positions
    const T *sb_val = nullptr;
    T *t = nullptr;                     // [m] workspace: b2 - A21 u1
    T *y = nullptr;                     // [m] workspace
    T *xs = nullptr;                    // [nsep] workspace
    T *rs = nullptr;                    // [nsep] workspace: separator right-hand side
    int max_seg = 0;
};

}  // namespace mgc
