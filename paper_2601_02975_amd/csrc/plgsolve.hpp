// Precomputed exact solver of the PLG block A22 (eq. (5.6)).
#pragma once

#include <vector>

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

}  // namespace mgc
