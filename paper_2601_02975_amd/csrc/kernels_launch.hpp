// Host-side launchers of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace mgc {

// one block-smoother sweep (Definition 5.6), uold -> unew: launch A (SFV
// tiles, PLG gathers and segment solves), then launch B (separators and
// segment corrections; nothing on levels without separators);
// ev0/ev1 (may be null) take the start and end of the SFV tile kernel's
// execution (the whole launch A where it is one kernel)
template <typename T>
void launch_smooth_a(const LevelArgs &L, const T *uold, const T *b, T *unew, const uint8_t *mask, bool uzero,
                     const PlgDev<T> &P, hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
template <typename T>
void launch_smooth_b(const PlgDev<T> &P, T *unew, hipStream_t st);
// two block-smoother sweeps uold -> ub -> uc on a level whose launch A is
// split (LevelArgs::split_a, Jacobi): pairs[0, npair) are the tiles of
// split_tile_rows(sizeof(T)) rows (row-major tile numbers, 64 cells wide)
// whose cells and 2-cell halo are SFV cells and whose 4-cell halo lies in
// the box, singles[0, nsingle) the other tiles with SFV cells; ev0/ev1 (may
// be null) take the start and end of the first kernel's execution (the
// two-sweep tiles)
template <typename T>
void launch_smooth_pair(const LevelArgs &L, const T *uold, const T *b, T *ub, T *uc, const uint8_t *mask,
                        bool uzero, const PlgDev<T> &P, const int *pairs, int npair, const int *singles, int nsingle,
                        hipStream_t st, hipEvent_t ev0, hipEvent_t ev1);
template <typename T>
void launch_fill_zero(size_t n, T *u, hipStream_t st);
template <typename T>
void launch_plg_residual(int m, const int *cell, const int *ptr, const int *col, const T *val, const T *b,
                         const T *u, T *r, hipStream_t st);
// u == nullptr: restrict b itself (FMG), else the residual b - A u
template <typename T>
void launch_restrict(const LevelArgs &L, const LevelArgs &C, const T *u, const T *b, const uint8_t *mask,
                     const int *plgidx, const T *rplg, const uint8_t *rmask, T *bc, T *uc, int nt, const int *ex_ptr,
                     const int *ex_target, const int *ex_child, bool skip_dead, hipStream_t st);
// set: u = P ec (FMG), else u += P ec
template <typename T>
void launch_prolong(const LevelArgs &L, const LevelArgs &C, const uint8_t *mask, const uint8_t *cmask, const T *ec,
                    T *u, int nex, const int *ex_fine, const int *ex_coarse, bool set, hipStream_t st);
template <typename TI, typename TO>
void launch_bottom(int n, const int *cells, const double *ainv, const TI *b, TO *x, hipStream_t st);
// residual b - A u (u + e when e is given, FP32 or FP64 (e64), written to
// uout) with partial
// max-norms per block; returns the number of blocks
int launch_residual_norm(const LevelArgs &L, const double *u, const void *e, bool e64, double *uout, const double *b,
                         const uint8_t *mask, int m, const int *pcell, const int *fe_col, const double *fe_val,
                         float *r32, double *r64, double *partial, hipStream_t st);
// number of partial maxima launch_residual_norm writes on a level with m PLG rows
int residual_norm_blocks(const LevelArgs &L, int m);
// capacity, in doubles, of the fixed device scratch of the no-allocation
// entry point; noalloc_scratch() returns its address on the current device
// (resolved once per device with hipGetSymbolAddress), or null on failure
constexpr int NOALLOC_SCRATCH_DOUBLES = 32768;
double *noalloc_scratch();
void launch_absmax(int n, const double *v, const uint8_t *mask, double *partial, int nblocks, hipStream_t st);
void launch_rhs(size_t n, const uint8_t *mask, const double *f, double *b, int nrows, const int *ptr, const int *cell,
                const int *gidx, const double *coef, const double *g, hipStream_t st);
void launch_zero_inactive(size_t n, const uint8_t *mask, double *u, hipStream_t st);
// one Gauss-Jordan step (pivot column k) on the augmented n x 2n array W
// (row-major, [A | I] at the start); f holds n multipliers, status one int
// (0 on entry)
void launch_gj_step(int n, int k, double *W, double *f, int *status, double tiny, hipStream_t st);
void launch_fit(int m, const double *M, const double *phi, const double *w, const int *ncol, double *work,
                double *beta, int *status, hipStream_t st);

}  // namespace mgc
