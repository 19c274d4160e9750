// Internal host-side structures of the cut-cell multigrid library.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "mg.h"

namespace mgc {

struct status_error : std::runtime_error {
    mg_status code;
    status_error(mg_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(mg_status c, const std::string &m) { throw status_error(c, m); }

constexpr int NB = 15;                 // dim Pi_4^2
extern const int MONO_P[NB];           // exponents of x in the basis order
extern const int MONO_Q[NB];           // exponents of y
int mono_index(int p, int q);

struct Seg {
    int kind;        // MG_SEG_LINE / MG_SEG_ARC / MG_SEG_CUBIC
    double p[8];
    int bc;
    double al1, al2;
    void point(double t, double &x, double &y) const;
    void deriv(double t, double &dx, double &dy) const;
};

struct BPiece { int curve, seg; double ta, tb; };

// one item of a component's boundary loop (used for cell quadrature)
struct LoopItem {
    int is_edge;          // 0: curve piece, 1: perimeter piece
    BPiece piece;         // curve piece
    int side;             // perimeter piece: 0 bottom, 1 right, 2 top, 3 left
    double s0, s1;        // position along the side, counter-clockwise
};

struct FacePiece { int64_t key; double lo, hi; };

struct Comp {
    int ci, cj;                       // grid cell
    bool full;                        // the whole grid cell
    double mom[NB];                   // ∬ X^p Y^q about the cell centre, X = (x - xc)/h
    std::vector<FacePiece> faces;
    std::vector<BPiece> bp;
    std::vector<LoopItem> items;
    double key;                       // order within the cell
    int parent;                       // union-find
    std::vector<int> absorbed;
    double vtot;                      // volume (h^2 units) of the region rooted here
};

struct CellData {                      // an irregular active cell
    double mom[NB];                   // about the centre of its own grid cell
    std::vector<BPiece> bp;
    std::vector<int> members;         // component ids
};

// Cut cells of one grid after Algorithm 1.
struct CutGrid {
    mg_grid g;
    double eps;
    int box_bc[4];                    // bottom, right, top, left
    double box_al[4][2];              // Robin (alpha1, alpha2) of the box sides
    std::vector<uint8_t> active, regular;     // [j*nx + i]
    std::vector<double> volfrac;
    std::vector<Comp> comps;
    std::vector<int> irr_cells;               // cell indices with CellData, row-major
    std::vector<CellData> irr;                // parallel to irr_cells
    std::vector<int> irr_slot;                // [j*nx+i] -> index into irr or -1
    std::vector<int> owner;                   // [j*nx+i] -> owner cell of removed cells or -1
    std::vector<Seg> const *curves_flat = nullptr;
};

struct Curves {
    std::vector<std::vector<Seg>> c;  // c[0] = box
};

void build_cutgrid(const Curves &cv, const mg_grid &g, double eps, CutGrid &out);
void cell_moments(const CutGrid &cg, int i, int j, double mom[NB]);
void full_moments(double mom[NB]);
void shift_moments(const double *m, int dx, int dy, double *out);

// Gauss-Legendre nodes/weights on [-1, 1]
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);

}  // namespace mgc
