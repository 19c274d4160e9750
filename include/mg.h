/*
 * mg.h -- C ABI of the MI355X cut-cell multigrid library.
 *
 * Solves a u_xx + b u_xy + c u_yy = f in Omega, N u = g on dOmega
 * (Section 1, eqs. (1.1)-(1.2); b^2 - 4ac < 0) with the fourth-order
 * finite-volume cut-cell discretisation (Section 4) and the cut-cell V-cycle
 * with the block smoother (Section 5, Definition 5.6, Algorithm 3).
 *
 * Conventions
 *  - Omega is the grid box minus holes.  curves[0] must be the grid box
 *    itself, counter-clockwise, one line segment per side (bottom, right,
 *    top, left), each carrying the boundary condition of that side
 *    (Dirichlet, Neumann or Robin; the Robin ghost cells are the degree-4
 *    reconstruction of Section 4.1 with the Robin condition at the face).
 *    curves[1..] are holes made of line segments, circular arcs and cubic
 *    Bezier pieces, closed, clockwise (Omega on the left, Section 2),
 *    strictly inside the box.
 *  - Cell arrays (f, u, b, r) are row-major with a halo of 2 cells on each
 *    side: cell (i, j), 0 <= i < nx, 0 <= j < ny, lives at index
 *    (j + 2) * (nx + 4) + (i + 2).  Entries of inactive cells (outside
 *    Omega or merged into a neighbour, Algorithm 1) and of the halo are
 *    ignored on input and written as 0 on output.
 *  - f holds cell averages <f>_i over the cut cells (eq. (4.1)), not point
 *    values.  g holds boundary averages (eq. (4.2)) in the layout returned
 *    by mg_boundary_quadrature: first the 2nx + 2ny box faces (bottom faces
 *    i = 0..nx-1, then top faces, then left faces j = 0..ny-1, then right
 *    faces; Dirichlet: average of u, Neumann: average of du/dn with n the
 *    outward normal), then one value per irregular cut cell, <<N u>> over
 *    its cut boundary B_i.
 *  - Pointers named *_dev are device pointers (HIP), owned by the caller,
 *    valid on the device the handle was created on.  Every call is ordered
 *    on the HIP stream `stream` (NULL = the null stream); calls that return
 *    host scalars synchronise that stream before returning.
 *  - A handle owns all of its device memory and must not be used from two
 *    host threads at once.
 *  - Every entry point returns an mg_status; MG_OK is 0.  On error nothing
 *    is written to outputs except where stated.
 */
#ifndef MG_H
#define MG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mg_handle_s *mg_handle;

typedef enum {
    MG_OK = 0,
    MG_ERR_INVALID_ARG = -1,   /* bad pointer, size, coefficient or option */
    MG_ERR_GEOMETRY = -2,      /* the grid does not resolve the geometry (Algorithm 1
                                  precondition), or no poised lattice exists */
    MG_ERR_SINGULAR = -3,      /* a dense factorisation met a zero pivot */
    MG_ERR_NO_CONVERGENCE = -4,/* max_iters reached; u holds the last iterate */
    MG_ERR_DIVERGED = -5,      /* residual grew for 3 iterations or became NaN */
    MG_ERR_OOM = -6,           /* device allocation failed */
    MG_ERR_HIP = -7,           /* a HIP runtime call failed */
    MG_ERR_UNSUPPORTED = -8    /* e.g. a PLG row wider than the kernels' row width, a coarsest
                                  level too large for the dense bottom solve */
} mg_status;

/* MG_BC_PERIODIC: box sides only, in opposite pairs (left and right, or
 * bottom and top; Sec. 4.1): a ghost position beyond such a side is the cell
 * one period away, and the side carries no data (its entries of g are
 * ignored). */
typedef enum { MG_BC_DIRICHLET = 0, MG_BC_NEUMANN = 1, MG_BC_ROBIN = 2, MG_BC_PERIODIC = 3 } mg_bc;
typedef enum { MG_SEG_LINE = 0, MG_SEG_ARC = 1, MG_SEG_CUBIC = 2 } mg_seg_kind;

/* One boundary segment.  LINE: p = {x0, y0, x1, y1}; ARC: p = {cx, cy, r,
 * theta0, theta1} with signed sweep theta1 - theta0; CUBIC: a cubic Bezier
 * piece (the spline boundaries of Section 2), p = {x0, y0, x1, y1, x2, y2,
 * x3, y3} its control points.  bc with the Robin coefficients: N u =
 * alpha1 u + alpha2 du/dn (eq. (1.2)).  Unused entries of p are ignored. */
typedef struct {
    int kind;
    double p[8];
    int bc;
    double alpha1, alpha2;
} mg_segment;

typedef struct { int n_seg; const mg_segment *seg; } mg_curve;

/* Finest grid: cells (x0 + i h, x0 + (i+1) h) x (y0 + j h, y0 + (j+1) h). */
typedef struct { double x0, y0, h; int nx, ny; } mg_grid;

typedef enum { MG_FP64 = 0, MG_MIXED = 1 } mg_precision;

/* Outer iteration of mg_solve: V-cycles (Algorithm 3), or FMG cycles
 * (Algorithm 4) on the residual equation, u <- u + FMG(b - A u) (Sec. 5.4). */
typedef enum { MG_CYCLE_V = 0, MG_CYCLE_FMG = 1 } mg_cycle;

typedef enum { MG_SMOOTH_JACOBI = 0, MG_SMOOTH_MULTICOLOUR = 1 } mg_colouring;

typedef struct {
    double eps;        /* volume-fraction threshold of Algorithm 1 (default 0.08) */
    double omega;      /* Jacobi weight of eq. (5.5) (default 0.5) */
    int nu1, nu2;      /* pre/post smoothing sweeps of Algorithm 3 (default 3, 3) */
    int n_levels;      /* 0 = coarsen while the coarser grid is valid and >= min_coarse cells per side */
    int min_coarse;    /* default 16 */
    int precision;     /* mg_precision (default MG_FP64) */
    int max_iters;     /* outer iterations of mg_solve (default 100) */
    int cycle;         /* mg_cycle (default MG_CYCLE_V) */
    int degree;        /* degree n of the PLG fits, Sec. 4.2 (default 4: lattices of 15 cells;
                          other values return MG_ERR_UNSUPPORTED) */
    double w_min;      /* smallest weight of eq. (4.17): W^{-1} = diag(max(|d_k|, w_min)), and the
                          weight of the boundary term (default 0.5) */
    int colouring;     /* mg_colouring of the SFV half of the smoother (default MG_SMOOTH_JACOBI, the
                          omega-Jacobi of eq. (5.5); MG_SMOOTH_MULTICOLOUR is an extension, see
                          mg_setup) */
    /* Launch shapes of the smoother (0 = the library's choice by grid size;
     * they change timing only, never results): levels with at least
     * split_cells cells run the SFV tiles and the PLG groups of launch A as
     * two kernels (default 2048^2; 1 = every level); levels with at most
     * small_cells cells use 8-row tiles in the fused kernel (default 512^2
     * in FP32, 256^2 in FP64; -1 = never); levels with at least split_b_sep
     * separator unknowns run launch B as two kernels (default 768; 1 =
     * every level with separators). */
    long long split_cells, small_cells;
    int split_b_sep;
    /* Partition of the PLG block solve (0 = the library's choice): hole
     * chains of at most seg_whole PLG cells are solved by one dense inverse
     * (default 768); longer chains are cut into segments of at most seg_max
     * cells (32..768, default 256) coupled through separator unknowns.  Any
     * partition solves A22 exactly; it changes the rounding and the timing. */
    int seg_max, seg_whole;
    /* Two-sweep tiles (0 = on, -1 = off; timing, and rounding only): on
     * levels whose launch A is split, with the Jacobi smoother, consecutive
     * sweeps are run in pairs, and the tiles whose cells and 2-cell halo are
     * SFV cells and whose 4-cell halo lies inside the box do both sweeps'
     * SFV updates in one pass (eq. (5.5) twice: the PLG block solve between
     * the sweeps does not reach them). */
    int pair_sweeps;
} mg_options;

typedef struct {
    int n_levels;
    int nx[16], ny[16];
    int n_active[16];          /* cut cells in C^h_eps per level */
    int n_plg[16];             /* PLG cells per level (Definition 4.1) */
    int n_sep[16];             /* separator unknowns of the PLG block solve per level */
    long long sweep_words[16]; /* algorithmic words moved by the first launch of one smoother
                                  sweep per level: u, b read and u written on every SFV cell,
                                  every PLG segment inverse read once, b read and u (or the
                                  segment solution) written on every PLG row; times the word
                                  size (8 FP64, 4 FP32), plus nx*ny bytes of the class mask */
    long long n_sfv[16];       /* SFV cells per level */
    int n_face, n_irr;         /* boundary-data layout sizes (finest level) */
    long long nnz_plg;         /* nonzeros of the PLG rows, all levels */
    long long device_bytes;    /* device memory held by the handle */
    double setup_seconds;      /* wall time of mg_setup */
    double cond_A22[16];       /* 1-norm condition number of A22 per level (Hager's estimate, a
                                  lower bound that is usually exact; 0 without PLG cells) */
    /* wall time of the setup stages, summed over levels (cf. Table 6):
     * [0] cut cells and merging (Algorithm 1), [1] classification and
     * lattices, [2] moments and the fits of the linear system, [3] the PLG
     * block solver (ordering, factors) and its device layout, [4] the bottom
     * inverse, [5] everything else (uploads, right-hand-side tables) */
    double setup_stage_seconds[6];
    long long n_pair_sfv[16];  /* SFV cells in two-sweep tiles per level (see pair_sweeps) */
} mg_info;

/* Defaults listed in mg_options. */
mg_status mg_default_options(mg_options *opt);

/* Builds the level hierarchy (eq. (5.7)): on every level the cut cells and
 * Algorithm 1, the SFV/PLG classification (Definition 4.1), the poised
 * lattices and the weighted minimum-norm fits (eqs. (4.10)-(4.18), computed
 * in FP64 on the GPU), the PLG block solver and the bottom-level inverse.
 * opt may be NULL (defaults).  On success *out owns the device data. */
mg_status mg_setup(const mg_grid *grid, int n_curves, const mg_curve *curves,
                   double a, double b, double c, const mg_options *opt,
                   void *stream, mg_handle *out);

/* Outer iteration: b = f - N g (eq. (4.19)), then V-cycles (Algorithm 3;
 * in MG_MIXED precision an FP32 V-cycle on the FP64 residual, added in FP64)
 * until ||b - A u||_inf <= tol ||b||_inf or max_iters.  u_dev is the initial
 * guess on entry and the solution on exit.  *iters and *rel_residual are
 * written on MG_OK, MG_ERR_NO_CONVERGENCE and MG_ERR_DIVERGED (the residual
 * grew three times in a row or is not finite; u holds the last iterate). */
mg_status mg_solve(mg_handle h, const double *f_dev, const double *g_dev, double *u_dev,
                   double tol, void *stream, int *iters, double *rel_residual);

/* b_dev = f - N g on the finest level (eq. (4.19)). */
mg_status mg_rhs(mg_handle h, const double *f_dev, const double *g_dev, double *b_dev, void *stream);

/* One FP64 V-cycle (Algorithm 3) on A u = b, updating u_dev in place. */
mg_status mg_vcycle(mg_handle h, const double *b_dev, double *u_dev, void *stream);

/* One block-smoother sweep (Definition 5.6) on level `level`; u_dev, b_dev
 * use that level's padded layout (nx_l + 4 columns). */
mg_status mg_smooth(mg_handle h, int level, const double *b_dev, double *u_dev, void *stream);

/* The same sweep in FP32 (the smoother of the mixed-precision V-cycle). */
mg_status mg_smooth32(mg_handle h, int level, const float *b_dev, float *u_dev, void *stream);

/* Residual restriction of Algorithm 3 (eq. (5.8)): bc_dev (level + 1's
 * layout) = R (b - A u) on level `level`, every residual computed (also on
 * PLG rows); precision MG_FP64 (double arrays) or MG_MIXED (float arrays). */
mg_status mg_restrict(mg_handle h, int level, int precision, const void *b_dev, const void *u_dev, void *bc_dev,
                      void *stream);

/* Correction of Algorithm 3 (eq. (5.9)): u_dev (level `level`) += the
 * piecewise-constant interpolation of ec_dev (level + 1); precision as for
 * mg_restrict. */
mg_status mg_prolong(mg_handle h, int level, int precision, const void *ec_dev, void *u_dev, void *stream);

/* r_dev = b - A u on level `level` (r_dev may be NULL) and *rnorm = ||r||_inf
 * over active cells (rnorm may be NULL). */
mg_status mg_residual(mg_handle h, int level, const double *b_dev, const double *u_dev,
                      double *r_dev, double *rnorm, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops): the residual and its norm of mg_residual,
 * with the norm written to the device scalar *rnorm_dev instead of the host,
 * no synchronisation and no allocation of any kind.  The per-block partial
 * maxima go to a fixed array of 32768 doubles (256 KiB) in device memory that
 * the library holds on each device for the life of the process (enough for
 * grids of about 4 x 4096^2 cells); a level that needs more returns
 * MG_ERR_UNSUPPORTED.  Every call on one device shares that array: calls that
 * overlap on one device (other streams or threads) race and must be ordered
 * by the caller.  r_dev may be NULL. */
mg_status mg_residual_norm_noalloc(mg_handle h, int level, const double *b_dev, const double *u_dev, double *r_dev,
                                   double *rnorm_dev, void *stream);

mg_status mg_query(mg_handle h, mg_info *info);

/* Host copies of one level's structure: kind[ny*nx] (0 inactive, 1 SFV,
 * 2 PLG, row-major without halo; may be NULL), and the PLG rows of A in
 * CSR form over PLG cells in row-major cell order: row_ptr[n_plg + 1],
 * col[nnz] (row-major cell index j*nx + i), val[nnz]; beta_b[n_plg] holds
 * the boundary coefficient of irregular rows and 0 otherwise.  Call with
 * col == NULL to get *nnz only. */
mg_status mg_export_level(mg_handle h, int level, int *kind, int *n_plg, long long *nnz,
                          int *row_ptr, int *col, double *val, double *beta_b);

/* Quadrature rules that let callers form the inputs.
 * Cells: for every active cell that is not a full grid cell, nodes and
 * weights with sum_k w_k F(x_k, y_k) = <F> over the cut cell; full cells
 * take any rule of the caller's choosing.  Boundary: for every entry of g,
 * nodes, weights summing to 1 and the outward unit normal, so that
 * sum_k w_k (N u)(x_k, y_k) = g_entry (box faces use the face's own BC,
 * irregular cells the BC of the segment each node lies on: bc[k],
 * alpha1[k], alpha2[k]).  CSR layout: ptr[n + 1] offsets into the node
 * arrays.  Call with x == NULL to get the sizes (*n, *nnodes) only.
 * cell[k] (cells only) is the row-major cell index of entry k. */
mg_status mg_cell_quadrature(mg_handle h, int *n, long long *nnodes, int *cell, long long *ptr,
                             double *x, double *y, double *w);
mg_status mg_boundary_quadrature(mg_handle h, int *n, long long *nnodes, long long *ptr,
                                 double *x, double *y, double *w, double *nx, double *ny,
                                 int *bc, double *alpha1, double *alpha2);

/* Forms the inputs of mg_solve from functions of the caller (host side,
 * outside the solve; cf. eqs. (4.1)-(4.2)): f_dev receives the cell
 * averages <f>_i and g_dev the boundary averages of the data, in the layouts
 * of mg_solve.  The callbacks evaluate batches of n points:
 *   f(n, x, y, out, ctx): out[k] = f(x[k], y[k]);
 *   g(n, x, y, curve, seg, nx, ny, out, ctx): out[k] = the boundary datum
 *   (N u)(x[k], y[k]) on segment seg of curve curve (box faces: curve 0, seg =
 *   side 0 bottom, 1 right, 2 top, 3 left), (nx, ny) the outward unit normal.
 * Full cells use a gauss_points x gauss_points Gauss-Legendre rule (1..16,
 * exact for polynomials of degree 2 gauss_points - 1 in each variable); cut
 * cells and the boundary use the rules of mg_cell_quadrature and
 * mg_boundary_quadrature.  g may be NULL only when the layout of g is empty.
 * Synchronises `stream`. */
typedef void (*mg_f_batch)(long long n, const double *x, const double *y, double *out, void *ctx);
typedef void (*mg_g_batch)(long long n, const double *x, const double *y, const int *curve, const int *seg,
                           const double *nx, const double *ny, double *out, void *ctx);
mg_status mg_project_rhs(mg_handle h, mg_f_batch f, mg_g_batch g, void *ctx, int gauss_points, double *f_dev,
                         double *g_dev, void *stream);

mg_status mg_destroy(mg_handle h);
const char *mg_error_string(mg_status s);

/* Kernel timing for measurement: enable = 1 clears the record and makes
 * mg_solve launch its outer iterations eagerly (instead of replaying its
 * captured graphs) with a pair of HIP events that take the start and end of
 * the execution of every finest-level launch of the smoother's SFV tile kernel (the
 * dominant kernel: the omega-Jacobi sweep of eq. (5.5); on levels where
 * launch A is one kernel, that whole kernel; where sweeps run in pairs
 * (pair_sweeps), only the kernel of the two-sweep tiles, and sweeps left
 * over from the pairs are not recorded).  enable = 0 stops recording
 * and returns the number of recorded launches and their average duration in
 * milliseconds. */
mg_status mg_kernel_timing(mg_handle h, int enable, int *launches, double *avg_ms);

/* eager = 1 makes mg_solve launch its kernels one by one on the caller's
 * stream instead of replaying its captured HIP graphs (the same kernels and
 * arguments; for checking the graphs against eager launches); eager = 0
 * (the default) replays graphs. */
mg_status mg_set_eager(mg_handle h, int eager);

/* ---------------------------------------------------------------------------
 * Solve server (an extension; the paper has no serving layer).
 *
 * A persistent loop on one device that admits solve requests continuously:
 * requests wait in arrival order and are started as soon as one of
 * max_active slots is free, the request's problem is not already being
 * solved, and the problem's hierarchy fits in the device-memory budget
 * (hierarchies stay resident between requests; idle ones are evicted least
 * recently used first when a new one would exceed the budget).  Each slot
 * runs its solves on its own non-blocking HIP stream, so solves of different
 * requests overlap on the device.  The solve of a request is exactly
 * mg_solve on the problem's hierarchy: its result does not depend on what
 * else runs.
 *
 * A problem is the data of mg_setup (copied; its setup runs in a slot at
 * the first request).  Requests pass device pointers f_dev, g_dev, u_dev in
 * the layouts of mg_solve; they must stay valid, and must not be touched by
 * the caller, until the request is done.  u_dev holds the initial guess.
 * Calls are thread-safe.
 */
typedef struct mg_server_s *mg_server;

typedef struct {
    int max_active;            /* slots: solves in flight at once (>= 1) */
    long long hbm_budget;      /* device bytes the resident hierarchies may hold */
} mg_server_options;

typedef struct {
    long long submitted, completed, failed;
    double p50_latency_s, p99_latency_s;    /* submit -> done, completed requests */
    double p50_solve_s, p99_solve_s;        /* start -> done (setup of a new problem included) */
    double solves_per_s;                    /* completed / (last done - first submit) */
    long long resident_bytes;               /* device bytes of resident hierarchies */
    int resident_problems, evictions;
    double sweep_gbs;                       /* algorithmic HBM GB/s of the smoothing sweeps of the
                                               completed solves over the same span as solves_per_s:
                                               per outer iteration, nu1 + nu2 sweeps on every level
                                               above the bottom, each reading u and b and writing u
                                               on the SFV cells (3 words per cell) */
} mg_server_stats;

/* Starts the server on the calling thread's current device. */
mg_status mg_server_create(const mg_server_options *opt, mg_server *out);

/* Registers a problem (no device work yet); *problem is its id. */
mg_status mg_server_add_problem(mg_server s, const mg_grid *grid, int n_curves, const mg_curve *curves,
                                double a, double b, double c, const mg_options *opt, int *problem);

/* Queues a solve of problem `problem` to tolerance tol; *ticket names it. */
mg_status mg_server_submit(mg_server s, int problem, const double *f_dev, const double *g_dev, double *u_dev,
                           double tol, unsigned long long *ticket);

/* State of a request: *done = 1 once finished; then *status, *iters,
 * *rel_residual (as mg_solve returns them) and *latency_s (submit -> done)
 * are valid.  Any output pointer may be NULL.  wait blocks until done. */
mg_status mg_server_poll(mg_server s, unsigned long long ticket, int *done, mg_status *status, int *iters,
                         double *rel_residual, double *latency_s);
mg_status mg_server_wait(mg_server s, unsigned long long ticket, mg_status *status, int *iters,
                         double *rel_residual, double *latency_s);

/* Text of the failure of a finished request ("" if it succeeded or the
 * ticket is unknown); valid until mg_server_destroy. */
const char *mg_server_request_error(mg_server s, unsigned long long ticket);

mg_status mg_server_get_stats(mg_server s, mg_server_stats *stats);

/* Waits for all queued requests, then frees every resident hierarchy. */
mg_status mg_server_destroy(mg_server s);

/* Human-readable description of the last failure of any entry point on the
 * calling host thread ("" if none); valid until the next call. */
const char *mg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MG_H */
