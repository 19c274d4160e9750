// Host-side description of one multigrid level.
#pragma once

#include <array>
#include <map>
#include <utility>
#include <vector>

#include "mg_internal.hpp"

namespace mgc {

void ghost_weights(int bc, int which, double w[5]);
void face_ghost(int bc, double al1, double al2, double h, int which, double w[5]);
void corner_weights(const CutGrid &cg, int xside, int yside, int m, int k, double h, double wu[4][4], double wgy[4],
                    double wgx[4]);

struct Level {
    mg_grid g{};
    double a = 0, b = 0, c = 0;
    double w_min = 0.5;                           // smallest weight of eq. (4.17), boundary weight
    const Curves *curves = nullptr;
    CutGrid cg;
    std::vector<uint8_t> kind;                    // 0 inactive, 1 SFV, 2 PLG (row-major)
    std::vector<int> plg_cells;                   // PLG cells, row-major order
    std::vector<int> plg_row;                     // cell -> PLG row or -1
    std::vector<std::vector<std::array<int, 2>>> lattices;
    int n_active = 0, n_face = 0, n_irr = 0;
    std::vector<int> g_of_cell;                   // irregular cell -> index into g
    // assembled PLG rows (row-major PLG order): columns are cell indices
    std::vector<int> row_ptr, col;
    std::vector<double> val, beta_b;

    int face_index(int side, int k) const;
    void classify();
    __uint128_t lattice_key(int i, int j) const;
    std::vector<std::vector<std::array<int, 2>>> lattice_candidates(int i, int j) const;
    void fit_inputs(std::vector<double> &M, std::vector<double> &phi, std::vector<double> &w, std::vector<int> &ncol);
    void sfv_row(int i, int j, std::vector<std::pair<int, double>> &cells,
                 std::vector<std::pair<int, double>> &gdat) const;
};

}  // namespace mgc
