// Precomputed exact solver of the PLG block A22 (eq. (5.6)).
#pragma once

#include <vector>

#include "kernels.hpp"
#include "level.hpp"

namespace mgc {

struct PlgSolver {
    int m = 0;                       // PLG unknowns
    std::vector<int> order;          // solve position -> PLG row (row-major PLG order)
    int nseg = 0;
    std::vector<int> seg_start;      // nseg + 1 positions
    int nsep = 0, sep_begin = 0;     // separators occupy positions [sep_begin, m)
    std::vector<long long> inv_off;  // segment inverses, row-major
    std::vector<double> inv;
    std::vector<long long> f_off;    // F_j = B_j^{-1} A_{j,S}, row-major (L_j x k_j)
    std::vector<double> F;
    std::vector<int> fcols_ptr, fcols;   // separator columns of F_j
    std::vector<double> sinv;        // (S')^{-1}, row-major nsep x nsep
    std::vector<int> sb_ptr, sb_col; // separator rows: couplings to segment positions
    std::vector<double> sb_val;
};

void build_plg_solver(const Level &L, int seg_max, PlgSolver &S);

// 1-norm condition number ||A22||_1 ||A22^{-1}||_1 of the PLG block, the
// second factor by Hager's estimator in Higham's form (a lower bound, exact
// in most cases) from exact solves with A22 and its transpose through the
// solver's factors; 0 when there are no PLG cells.
double cond1_estimate(const Level &L, const PlgSolver &S);

// Work layout of the two smoother launches on the GPU.
//
// Launch A computes, per "group" of PLG rows (each segment is a group; the
// separator rows form groups of at most sep_group rows), the Jacobi-updated
// values of the SFV cells that the group's rows couple to (the set H of the
// group), then t = b2 - A21 u1 of the group's rows, and for a segment
// y = B^{-1} t on a slice of at most `slice` rows per block.  Launch B forms
// the separator right-hand side, solves with the Schur complement and
// corrects the segments.  Row-wise sparse data are stored with a fixed width
// of ELL_W entries per row (zero padding) so that a row's loads issue
// together.
struct PlgPlan {
    int ngroup = 0;
    std::vector<int> grp_start;              // ngroup + 1 solve positions
    std::vector<int> hptr, hcell;            // H of each group: padded cell indices
    std::vector<int> a21_loc;                // [m * ELL_W] index into H of the row's group
    std::vector<double> a21_val;             // [m * ELL_W]
    std::vector<PlgBlkA> blk1;               // launch A PLG blocks
    std::vector<PlgBlkB> blk2;               // launch B blocks
    // A_SB: entry k of separator row s is slot s * ELL_W + k; per segment the
    // entries on its rows: (solve position of the row, slot, value)
    std::vector<int> ce_ptr, ce_row, ce_slot;
    std::vector<double> ce_val;
    std::vector<long long> ft_off;           // F_j^T, row-major k_j x L_j
    std::vector<double> FT;
    // dense blocks with rows padded to a multiple of 4 columns (zeros), for
    // 16-byte vector loads: segment inverses (L_j x pad4(L_j)), S'^{-1}
    // (nsep x pad4(nsep)) and its rows at the separator columns of F_j
    // (k_j x pad4(nsep))
    std::vector<long long> inv_off;
    std::vector<double> INV, SINV;
    std::vector<long long> sj_off;
    std::vector<double> SJ;
    int hmax = 0, lmax = 0, kmax = 0;
};

void build_plg_plan(const Level &L, const PlgSolver &S, int nx, int slice, int bslice, int sep_group,
                    int sep_rows, PlgPlan &P);

}  // namespace mgc
