// C ABI of the cut-cell multigrid library: setup orchestration, device data,
// the V-cycle driver (Algorithm 3) and the outer iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>

#include "kernels_launch.hpp"
#include "level.hpp"
#include "mg.h"
#include "plgsolve.hpp"

using namespace mgc;

namespace {

#define HIPCHECK(x)                                                                             \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess) fail(MG_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Device-wide synchronising work (allocation, frees, synchronous copies of
// setup and destruction) must not overlap a stream capture in another
// thread: both take this lock.
std::mutex g_capture_mu;

constexpr int SEG_MAX = 256;       // longest PLG segment (dense inverse per segment)
constexpr int SEG_WHOLE = 768;     // a level whose hole chains fit in segments this long needs no separators
constexpr int ITER_CHUNK = 8;      // most outer iterations per launch (chunks of 1, 2, 4, 8)
constexpr int BOTTOM_MAX = 4096;   // largest dense bottom inverse (128 MiB; right-hand side staged in 32 KiB of LDS)

struct DevLevel {
    LevelArgs args{};
    size_t ncells = 0;
    uint8_t *mask = nullptr;
    int *plgidx = nullptr;
    // iterates: two buffers, three on levels with two-sweep tiles
    double *u64[3] = {nullptr, nullptr, nullptr}, *b64 = nullptr, *rplg64 = nullptr;
    float *u32[3] = {nullptr, nullptr, nullptr}, *b32 = nullptr, *rplg32 = nullptr;
    int nbuf = 2;
    // two-sweep tiles and the other tiles with SFV cells (row-major tile
    // numbers of the split launch's tiles in the handle's cycle precision)
    int *pair_tiles = nullptr, *single_tiles = nullptr;
    int npair = 0, nsingle = 0, pair_word = 0;     // pair_word: the word size the lists are for
    long long n_pair_sfv = 0;
    int m = 0;
    int *plg_cell = nullptr, *full_ptr = nullptr, *full_col = nullptr;
    int *fe_col = nullptr;                  // PLG rows, fixed width (ELL_W), padded cell index
    double *fe_val = nullptr;
    double *full_val64 = nullptr;
    float *full_val32 = nullptr;
    PlgDev<double> P64;
    PlgDev<float> P32;
    int ex_nt = 0;                                                      // restriction to the next level:
    int *ex_ptr = nullptr, *ex_target = nullptr, *ex_child = nullptr;   // coarse cells with extra children
    uint8_t *rmask = nullptr;                                           // next level: 0 off, 1 tile, 2 extra list
    int pex_n = 0;
    int *pex_fine = nullptr, *pex_coarse = nullptr;                     // prolongation from the next level
    int nbot = 0;
    int *bot_cells = nullptr;
    double *ainv = nullptr;
    int cur = 0;
    long long sweep_words = 0;    // words moved by one smoother launch A (algorithmic)
    long long nsfv = 0;
    // finest level, FP64 FMG: residual equation right-hand side and its iterate
    double *r64 = nullptr, *e64[3] = {nullptr, nullptr, nullptr};
};

}  // namespace

struct mg_handle_s {
    int device = 0;
    mg_options opt{};
    double a = 0, b = 0, c = 0;
    Curves curves;
    std::vector<std::unique_ptr<Level>> levels;
    std::vector<PlgSolver> solvers;
    std::vector<DevLevel> dev;
    int nrhs = 0;
    int *rhs_ptr = nullptr, *rhs_cell = nullptr, *rhs_gidx = nullptr;
    double *rhs_coef = nullptr;
    double *partial = nullptr, *host_scalar = nullptr, *host_scalar_dev = nullptr;   // mapped host memory
    int npartial = 0;
    std::vector<void *> allocs;
    long long bytes = 0;
    double setup_seconds = 0.0;
    std::string last_error;
    // captured outer iteration per precision (0 FP64, 1 mixed)
    hipStream_t cap_stream = nullptr;
    // [FP64 | mixed from u64[0] | mixed from u64[1]] x [1, 2, 4, 8 iterations]
    hipGraphExec_t iter_exec[3][4] = {};
    hipGraph_t iter_graph[3][4] = {};
    int upar = 0;                 // mixed precision: which FP64 buffer holds the iterate
    // timing of the finest-level SFV tile kernel: in timing mode the outer
    // iterations are launched eagerly, each such launch with an event pair
    // that takes the start and end of its execution, read after each
    // synchronisation
    bool timing = false;
    std::vector<hipEvent_t> ev;          // pool, 2 per recorded launch of one graph
    int ev_next = 0;                     // next free pair while capturing
    int tim_last = 0;                    // pairs recorded by the last replay, not yet read
    bool tim_capture = false;
    bool eager = false;                  // mg_set_eager: launch instead of replaying graphs
    int nrec = 0;
    double tim_total_ms = 0.0;
    std::vector<double> cond_a22;
    double stage[6] = {0, 0, 0, 0, 0, 0};
    double *scratch = nullptr;           // the device's fixed scratch (mg_residual_norm_noalloc)

    template <typename T>
    T *alloc(size_t n) {
        if (n == 0) n = 1;
        void *p = nullptr;
        if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) fail(MG_ERR_OOM, "device allocation failed");
        HIPCHECK(hipMemset(p, 0, n * sizeof(T)));
        allocs.push_back(p);
        bytes += (long long)(n * sizeof(T));
        return (T *)p;
    }
    template <typename T>
    T *upload(const std::vector<T> &v) {
        T *p = alloc<T>(v.size());
        if (!v.empty()) HIPCHECK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
        return p;
    }
    template <typename T>
    T *upload_f32(const std::vector<double> &v) {
        std::vector<float> f(v.begin(), v.end());
        return upload(f);
    }
};

namespace {

size_t padded_index(int nx, int cell) { return (size_t)(cell / nx + 2) * (nx + 4) + (cell % nx + 2); }

LevelArgs make_args(const Level &L, const mg_options &o) {
    const double omega = o.omega;
    LevelArgs a{};
    a.nx = L.g.nx;
    a.ny = L.g.ny;
    a.pitch = L.g.nx + 4;
    a.h = L.g.h;
    double h2 = L.g.h * L.g.h;
    a.cxx = L.a / h2;
    a.cxy = L.b / h2;
    a.cyy = L.c / h2;
    a.omega_over_d = omega / (-2.5 * (L.a + L.c) / h2);
    a.mixed = L.b != 0.0;
    const long long cells = (long long)L.g.nx * L.g.ny;
    a.split_a = cells >= (o.split_cells > 0 ? o.split_cells : 2048LL * 2048) ? 1 : 0;
    a.small32 = o.small_cells < 0 ? 0 : cells <= (o.small_cells > 0 ? o.small_cells : 512LL * 512) ? 1 : 0;
    a.small64 = o.small_cells < 0 ? 0 : cells <= (o.small_cells > 0 ? o.small_cells : 256LL * 256) ? 1 : 0;
    a.colouring = o.colouring == MG_SMOOTH_MULTICOLOUR ? 1 : 0;
    a.periodic = (L.cg.box_bc[1] == MG_BC_PERIODIC ? 1 : 0) | (L.cg.box_bc[0] == MG_BC_PERIODIC ? 2 : 0);
    return a;
}

// batched weighted minimum-norm fits on the GPU, then the PLG rows
void fit_level(mg_handle h, Level &L, hipStream_t st) {
    std::vector<double> M, phi, w;
    std::vector<int> ncol;
    auto t0 = std::chrono::steady_clock::now();
    L.fit_inputs(M, phi, w, ncol);
    auto t1 = std::chrono::steady_clock::now();
    h->stage[1] += std::chrono::duration<double>(t1 - t0).count();
    struct StageClock {
        double &acc;
        std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
        ~StageClock() { acc += std::chrono::duration<double>(std::chrono::steady_clock::now() - t).count(); }
    } fit_clock{h->stage[2]};
    const int m = (int)L.plg_cells.size();
    L.row_ptr.assign(m + 1, 0);
    L.col.clear();
    L.val.clear();
    L.beta_b.assign(m, 0.0);
    if (m == 0) return;
    std::lock_guard<std::mutex> lk(g_capture_mu);
    double *dM, *dphi, *dw, *dwork, *dbeta;
    int *dncol, *dstat;
    HIPCHECK(hipMalloc(&dM, M.size() * 8));
    HIPCHECK(hipMalloc(&dphi, phi.size() * 8));
    HIPCHECK(hipMalloc(&dw, w.size() * 8));
    HIPCHECK(hipMalloc(&dncol, ncol.size() * 4));
    HIPCHECK(hipMalloc(&dwork, (size_t)m * 511 * 8));
    HIPCHECK(hipMalloc(&dbeta, (size_t)m * 16 * 8));
    HIPCHECK(hipMalloc(&dstat, (size_t)m * 4));
    HIPCHECK(hipMemcpy(dM, M.data(), M.size() * 8, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(dphi, phi.data(), phi.size() * 8, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(dw, w.data(), w.size() * 8, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(dncol, ncol.data(), ncol.size() * 4, hipMemcpyHostToDevice));
    launch_fit(m, dM, dphi, dw, dncol, dwork, dbeta, dstat, st);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(st));
    std::vector<double> beta((size_t)m * 16);
    std::vector<int> stat(m);
    HIPCHECK(hipStreamSynchronize(st));
    HIPCHECK(hipMemcpy(beta.data(), dbeta, beta.size() * 8, hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(stat.data(), dstat, stat.size() * 4, hipMemcpyDeviceToHost));
    (void)hipFree(dM); (void)hipFree(dphi); (void)hipFree(dw); (void)hipFree(dncol); (void)hipFree(dwork); (void)hipFree(dbeta); (void)hipFree(dstat);
    const int nx = L.g.nx;
    for (int r = 0; r < m; ++r) {
        if (!stat[r]) fail(MG_ERR_SINGULAR, "a PLG fit has a rank-deficient sample matrix");
        int cell = L.plg_cells[r];
        for (int k = 0; k < NB; ++k) {
            L.col.push_back(cell + L.lattices[r][k][1] * nx + L.lattices[r][k][0]);
            L.val.push_back(beta[(size_t)r * 16 + k]);
        }
        if (ncol[r] == NB + 1) L.beta_b[r] = beta[(size_t)r * 16 + NB];
        L.row_ptr[r + 1] = (int)L.col.size();
    }
}

// dense inverse of a row-major n x n matrix on the GPU: Gauss-Jordan with
// partial pivoting (launch_gj_step), FP64; a pivot column whose largest
// entry is below 1e-13 of the matrix's largest entry is reported singular
std::vector<double> gpu_inverse(int n, const std::vector<double> &A, hipStream_t st) {
    const size_t ld = 2 * (size_t)n;
    std::vector<double> W((size_t)n * ld, 0.0);
    double amax = 0.0;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) {
            const double v = A[(size_t)i * n + j];
            if (!std::isfinite(v)) fail(MG_ERR_SINGULAR, "the bottom-level matrix has a non-finite entry");
            W[(size_t)i * ld + j] = v;
            amax = std::max(amax, std::fabs(v));
        }
        W[(size_t)i * ld + n + i] = 1.0;
    }
    if (!(amax > 0.0)) fail(MG_ERR_SINGULAR, "the bottom-level matrix is zero");
    double *dW = nullptr, *df = nullptr;
    int *dstat = nullptr;
    auto release = [&]() {
        if (dW) (void)hipFree(dW);
        if (df) (void)hipFree(df);
        if (dstat) (void)hipFree(dstat);
    };
    try {
        HIPCHECK(hipMalloc(&dW, W.size() * 8));
        HIPCHECK(hipMalloc(&df, (size_t)n * 8));
        HIPCHECK(hipMalloc(&dstat, sizeof(int)));
        HIPCHECK(hipMemcpy(dW, W.data(), W.size() * 8, hipMemcpyHostToDevice));
        HIPCHECK(hipMemset(dstat, 0, sizeof(int)));
        for (int k = 0; k < n; ++k) launch_gj_step(n, k, dW, df, dstat, 1e-13 * amax, st);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipStreamSynchronize(st));
        int stat = 0;
        HIPCHECK(hipMemcpy(&stat, dstat, sizeof(int), hipMemcpyDeviceToHost));
        if (stat != 0) fail(MG_ERR_SINGULAR, "the bottom-level matrix is singular (pivot column " +
                                                 std::to_string(stat - 1) + ")");
        HIPCHECK(hipMemcpy(W.data(), dW, W.size() * 8, hipMemcpyDeviceToHost));
    } catch (...) {
        release();
        throw;
    }
    release();
    std::vector<double> out((size_t)n * n);
    for (int i = 0; i < n; ++i)
        std::copy(W.begin() + (size_t)i * ld + n, W.begin() + (size_t)(i + 1) * ld, out.begin() + (size_t)i * n);
    return out;
}

void upload_level(mg_handle h, int l, bool last, hipStream_t st) {
    Level &L = *h->levels[l];
    const PlgSolver &S = h->solvers[l];
    DevLevel &D = h->dev[l];
    const int nx = L.g.nx, ny = L.g.ny;
    D.args = make_args(L, h->opt);
    // ghost weights of the four box sides on this level (h-dependent for Robin)
    std::vector<double> gw(32);
    for (int side = 0; side < 4; ++side)
        for (int d = 1; d <= 2; ++d) {
            double w[5];
            face_ghost(L.cg.box_bc[side], L.cg.box_al[side][0], L.cg.box_al[side][1], L.g.h, d, w);
            for (int k = 0; k < 4; ++k) gw[(side * 2 + d - 1) * 4 + k] = w[k];
        }
    D.args.gw = h->upload(gw);
    // class flags of the blocks of 64 x 8 cells: every cell SFV; no SFV
    // cell; no active cell here nor among the 32 x 4 cells of the next level
    // under the block
    D.args.full_bx = (nx + 63) / 64;
    D.args.full_by = (ny + 7) / 8;
    std::vector<uint8_t> full((size_t)D.args.full_bx * D.args.full_by, 0);
    const Level *Cn = last ? nullptr : h->levels[l + 1].get();
    for (int by = 0; by < D.args.full_by; ++by)
        for (int bx = 0; bx < D.args.full_bx; ++bx) {
            bool all = bx * 64 + 64 <= nx && by * 8 + 8 <= ny, none = true, dead = true;
            for (int j = by * 8; j < std::min(by * 8 + 8, ny); ++j)
                for (int i = bx * 64; i < std::min(bx * 64 + 64, nx); ++i) {
                    const uint8_t k = L.kind[(size_t)j * nx + i];
                    all = all && k == 1;
                    none = none && k != 1;
                    dead = dead && k == 0;
                }
            if (dead && Cn)
                for (int j = by * 4; j < std::min(by * 4 + 4, Cn->g.ny); ++j)
                    for (int i = bx * 32; i < std::min(bx * 32 + 32, Cn->g.nx); ++i)
                        dead = dead && !Cn->cg.active[(size_t)j * Cn->g.nx + i];
            full[(size_t)by * D.args.full_bx + bx] =
                (uint8_t)((all ? FULL_ALL_SFV : 0) | (none ? FULL_NO_SFV : 0) | (dead ? FULL_DEAD : 0));
        }
    D.args.full = h->upload(full);
    // 64 x 32 tiles with an active cell here or on the next level under them
    {
        const int tiles_x = (nx + 63) / 64, tiles_y = (ny + 31) / 32;
        std::vector<int> live;
        for (int t = 0; t < tiles_x * tiles_y; ++t) {
            const int bx = t % tiles_x, by0 = (t / tiles_x) * 4;
            bool dead = true;
            for (int by = by0; by < std::min(by0 + 4, D.args.full_by); ++by)
                dead = dead && (full[(size_t)by * D.args.full_bx + bx] & FULL_DEAD);
            if (!dead) live.push_back(t);
        }
        if ((int)live.size() < tiles_x * tiles_y && !live.empty()) {
            D.args.live = h->upload(live);
            D.args.nlive = (int)live.size();
        }
    }
    D.ncells = (size_t)(nx + 4) * (ny + 4);
    std::vector<uint8_t> mask(D.ncells, 0);
    std::vector<int> plgidx(D.ncells, -1);
    for (int cell = 0; cell < nx * ny; ++cell) mask[padded_index(nx, cell)] = L.kind[cell];
    for (int q = 0; q < S.m; ++q) plgidx[padded_index(nx, L.plg_cells[S.order[q]])] = q;
    D.mask = h->upload(mask);
    D.plgidx = h->upload(plgidx);
    // two-sweep tiles (split launch A, Jacobi): all cells of the tile and
    // its 2-cell halo are SFV cells, and its 4-cell halo lies in the box
    if (D.args.split_a && !D.args.colouring && h->opt.pair_sweeps == 0) {
        const int word = h->opt.precision == MG_MIXED ? 4 : 8, tys = split_tile_rows(word);
        const int tiles_x = (nx + 63) / 64, tiles_y = (ny + tys - 1) / tys;
        std::vector<int> pairs, singles;
        for (int t = 0; t < tiles_x * tiles_y; ++t) {
            const int i0 = (t % tiles_x) * 64, j0 = (t / tiles_x) * tys;
            bool any = false;
            for (int j = j0; j < std::min(j0 + tys, ny); ++j)
                for (int i = i0; i < std::min(i0 + 64, nx); ++i) any = any || L.kind[(size_t)j * nx + i] == 1;
            if (!any) continue;
            bool pair = i0 >= 4 && i0 + 68 <= nx && j0 >= 4 && j0 + tys + 4 <= ny;
            for (int j = j0 - 2; pair && j < j0 + tys + 2; ++j)
                for (int i = i0 - 2; pair && i < i0 + 66; ++i) pair = L.kind[(size_t)j * nx + i] == 1;
            (pair ? pairs : singles).push_back(t);
        }
        if (!pairs.empty()) {
            D.npair = (int)pairs.size();
            D.nsingle = (int)singles.size();
            D.n_pair_sfv = (long long)D.npair * 64 * tys;
            D.pair_tiles = h->upload(pairs);
            D.single_tiles = h->upload(singles);
            D.nbuf = 3;
            D.pair_word = word;
        }
    }
    for (int k = 0; k < D.nbuf; ++k) {
        D.u64[k] = h->alloc<double>(D.ncells);
        D.u32[k] = h->alloc<float>(D.ncells);
    }
    D.b64 = h->alloc<double>(D.ncells);
    D.b32 = h->alloc<float>(D.ncells);
    // PLG rows in solve order
    D.m = S.m;
    std::vector<int> cell(S.m), fptr(S.m + 1, 0), fcol;
    std::vector<double> fval;
    for (int q = 0; q < S.m; ++q) {
        int r = S.order[q];
        cell[q] = (int)padded_index(nx, L.plg_cells[r]);
        for (int e = L.row_ptr[r]; e < L.row_ptr[r + 1]; ++e) {
            fcol.push_back((int)padded_index(nx, L.col[e]));
            fval.push_back(L.val[e]);
        }
        fptr[q + 1] = (int)fcol.size();
    }
    std::vector<int> fe_col((size_t)S.m * ELL_W);
    std::vector<double> fe_val((size_t)S.m * ELL_W, 0.0);
    for (int q = 0; q < S.m; ++q) {
        if (fptr[q + 1] - fptr[q] > ELL_W) fail(MG_ERR_UNSUPPORTED, "a PLG row is wider than the row width");
        for (int k = 0; k < ELL_W; ++k) {
            const int e = fptr[q] + k;
            fe_col[(size_t)q * ELL_W + k] = e < fptr[q + 1] ? fcol[e] : cell[q];
            if (e < fptr[q + 1]) fe_val[(size_t)q * ELL_W + k] = fval[e];
        }
    }
    D.fe_col = h->upload(fe_col);
    D.fe_val = h->upload(fe_val);
    D.plg_cell = h->upload(cell);
    D.full_ptr = h->upload(fptr);
    D.full_col = h->upload(fcol);
    D.full_val64 = h->upload(fval);
    D.full_val32 = h->upload_f32<float>(fval);
    D.rplg64 = h->alloc<double>(S.m);
    D.rplg32 = h->alloc<float>(S.m);
    PlgPlan G;
    auto p0 = std::chrono::steady_clock::now();
    build_plg_plan(L, S, nx, PLG_SLICE, PLG_B_ROWS, PLG_LMAX, PLG_SEP_ROWS, G);
    h->stage[3] += std::chrono::duration<double>(std::chrono::steady_clock::now() - p0).count();
    if (G.hmax > PLG_HMAX || G.lmax > PLG_LMAX || G.kmax > PLG_KMAX || S.nsep > PLG_SMAX)
        fail(MG_ERR_UNSUPPORTED, "PLG block partition exceeds the LDS staging limits on level " + std::to_string(l) +
                                     " (coupled SFV cells " + std::to_string(G.hmax) + "/" + std::to_string(PLG_HMAX) +
                                     ", group rows " + std::to_string(G.lmax) + "/" + std::to_string(PLG_LMAX) +
                                     ", separator columns " + std::to_string(G.kmax) + "/" + std::to_string(PLG_KMAX) +
                                     ", separators " + std::to_string(S.nsep) + "/" + std::to_string(PLG_SMAX) + ")");
    int *grp_start = h->upload(G.grp_start), *hptr = h->upload(G.hptr), *hcell = h->upload(G.hcell);
    int *a21_loc = h->upload(G.a21_loc);
    const PlgBlkA *blk1 = h->upload(G.blk1);
    const PlgBlkB *blk2 = h->upload(G.blk2);
    int *seg_start = h->upload(S.seg_start);
    long long *inv_off = h->upload(G.inv_off), *ft_off = h->upload(G.ft_off), *sj_off = h->upload(G.sj_off);
    int *fcols_ptr = h->upload(S.fcols_ptr);
    int *fcols = h->upload(S.fcols);
    int nblk2_seg = 0;
    for (auto &b : G.blk2) nblk2_seg += b.kind == 0 ? 1 : 0;
    int *ce_ptr = h->upload(G.ce_ptr), *ce_row = h->upload(G.ce_row), *ce_slot = h->upload(G.ce_slot);
    auto fill = [&](auto &P, auto *a21v, auto *inv, auto *cev, auto *FT, auto *SJ, auto *sinv, auto *t, auto *y,
                    auto *contrib) {
        P.m = S.m; P.nseg = S.nseg; P.nsep = S.nsep; P.sep_begin = S.sep_begin;
        P.cell = D.plg_cell;
        P.grp_start = grp_start; P.hptr = hptr; P.hcell = hcell;
        P.a21_loc = a21_loc; P.a21_val = a21v;
        P.nblk1 = (int)G.blk1.size(); P.blk1 = blk1;
        P.seg_start = seg_start; P.inv_off = inv_off; P.inv = inv;
        P.ce_ptr = ce_ptr; P.ce_row = ce_row; P.ce_slot = ce_slot; P.ce_val = cev;
        P.nblk2 = (int)G.blk2.size(); P.blk2 = blk2;
        P.ft_off = ft_off; P.FT = FT; P.fcols_ptr = fcols_ptr; P.sj_off = sj_off; P.SJ = SJ; P.sinv = sinv;
        P.fcols = fcols; P.nblk2_seg = nblk2_seg;
        P.split_b = S.nsep >= (h->opt.split_b_sep > 0 ? h->opt.split_b_sep : 768) ? 1 : 0;
        P.t = t; P.y = y; P.contrib = contrib;
    };
    const size_t nslot = (size_t)S.nsep * ELL_W;
    fill(D.P64, h->upload(G.a21_val), h->upload(G.INV), h->upload(G.ce_val), h->upload(G.FT), h->upload(G.SJ),
         h->upload(G.SINV), h->alloc<double>(S.m), h->alloc<double>(S.m), h->alloc<double>(nslot));
    fill(D.P32, h->upload_f32<float>(G.a21_val), h->upload_f32<float>(G.INV), h->upload_f32<float>(G.ce_val),
         h->upload_f32<float>(G.FT), h->upload_f32<float>(G.SJ), h->upload_f32<float>(G.SINV), h->alloc<float>(S.m),
         h->alloc<float>(S.m), h->alloc<float>(nslot));
    // algorithmic words of launch A: u, b read and u written on every SFV
    // cell, each segment inverse read once, b read and u (or y) written on
    // every PLG row
    long long nsfv = 0;
    for (int cl = 0; cl < nx * ny; ++cl) nsfv += L.kind[cl] == 1;
    D.sweep_words = 3 * nsfv + (long long)S.inv.size() + 2LL * S.m;
    D.nsfv = nsfv;
    // transfers to the next level
    if (!last) {
        const Level &C = *h->levels[l + 1];
        // fine cells whose coarse parent was merged away go to the cell that
        // absorbed it (restriction and prolongation)
        std::vector<std::pair<int, int>> ex;        // (coarse target cell, fine cell)
        for (int cellf = 0; cellf < nx * ny; ++cellf) {
            if (!L.cg.active[cellf]) continue;
            int ci = (cellf % nx) / 2, cj = (cellf / nx) / 2;
            int cc = cj * C.g.nx + ci;
            if (C.cg.active[cc]) continue;
            int own = C.cg.owner[cc];
            if (own < 0) fail(MG_ERR_GEOMETRY, "fine cell without a coarse parent");
            ex.push_back({own, cellf});
        }
        std::vector<int> pf, pc;
        for (auto &e : ex) {
            pf.push_back((int)padded_index(nx, e.second));
            pc.push_back((int)padded_index(C.g.nx, e.first));
        }
        // restriction: coarse cells with extra children take all their
        // children from a list (own active children first)
        std::vector<int> tg;
        for (auto &e : ex) tg.push_back(e.first);
        std::sort(tg.begin(), tg.end());
        tg.erase(std::unique(tg.begin(), tg.end()), tg.end());
        std::vector<uint8_t> rmask((size_t)(C.g.nx + 4) * (C.g.ny + 4), 0);
        for (int cc = 0; cc < C.g.nx * C.g.ny; ++cc) rmask[padded_index(C.g.nx, cc)] = C.cg.active[cc] ? 1 : 0;
        std::vector<int> ptr{0}, tgt, child;
        for (int t : tg) {
            rmask[padded_index(C.g.nx, t)] = 2;
            tgt.push_back((int)padded_index(C.g.nx, t));
            const int ci = t % C.g.nx, cj = t / C.g.nx;
            for (int q = 0; q < 4; ++q) {
                const int fi = 2 * ci + (q & 1), fj = 2 * cj + (q >> 1);
                if (fi < nx && fj < ny && L.cg.active[fj * nx + fi]) child.push_back((int)padded_index(nx, fj * nx + fi));
            }
            for (auto &e : ex)
                if (e.first == t) child.push_back((int)padded_index(nx, e.second));
            ptr.push_back((int)child.size());
        }
        D.ex_nt = (int)tgt.size();
        D.ex_ptr = h->upload(ptr);
        D.ex_target = h->upload(tgt);
        D.ex_child = h->upload(child);
        D.rmask = h->upload(rmask);
        D.pex_n = (int)pf.size();
        D.pex_fine = h->upload(pf);
        D.pex_coarse = h->upload(pc);
    } else {
        // bottom: dense inverse over the active cells
        std::vector<int> act, pos((size_t)nx * ny, -1);
        for (int cellc = 0; cellc < nx * ny; ++cellc)
            if (L.cg.active[cellc]) {
                pos[cellc] = (int)act.size();
                act.push_back(cellc);
            }
        const int n = (int)act.size();
        if (n > BOTTOM_MAX) fail(MG_ERR_UNSUPPORTED, "the coarsest level has too many cells for the dense bottom solve");
        std::vector<double> A((size_t)n * n, 0.0);
        std::vector<std::pair<int, double>> cells, gd;
        for (int r = 0; r < n; ++r) {
            int cl = act[r];
            if (L.kind[cl] == 1) {
                L.sfv_row(cl % nx, cl / nx, cells, gd);
                for (auto &e : cells) A[(size_t)r * n + pos[e.first]] += e.second;
            } else {
                int pr = L.plg_row[cl];
                for (int e = L.row_ptr[pr]; e < L.row_ptr[pr + 1]; ++e) A[(size_t)r * n + pos[L.col[e]]] += L.val[e];
            }
        }
        auto b0 = std::chrono::steady_clock::now();
        std::vector<double> inv = gpu_inverse(n, A, st);
        h->stage[4] += std::chrono::duration<double>(std::chrono::steady_clock::now() - b0).count();
        std::vector<int> bc(n);
        for (int r = 0; r < n; ++r) bc[r] = (int)padded_index(nx, act[r]);
        D.nbot = n;
        D.bot_cells = h->upload(bc);
        D.ainv = h->upload(inv);
    }
    (void)st;
}

void upload_rhs(mg_handle h) {
    const Level &L = *h->levels[0];
    const int nx = L.g.nx, ny = L.g.ny;
    std::vector<int> ptr{0}, cell, gidx;
    std::vector<double> coef;
    std::vector<std::pair<int, double>> cells, gd;
    for (int cl = 0; cl < nx * ny; ++cl) {
        std::map<int, double> acc;
        if (L.kind[cl] == 1) {
            L.sfv_row(cl % nx, cl / nx, cells, gd);
            for (auto &e : gd) acc[e.first] += e.second;
        } else if (L.kind[cl] == 2 && L.g_of_cell[cl] >= 0) {
            acc[L.g_of_cell[cl]] += L.beta_b[L.plg_row[cl]];
        }
        if (acc.empty()) continue;
        cell.push_back((int)padded_index(nx, cl));
        for (auto &kv : acc) {
            gidx.push_back(kv.first);
            coef.push_back(kv.second);
        }
        ptr.push_back((int)gidx.size());
    }
    h->nrhs = (int)cell.size();
    h->rhs_ptr = h->upload(ptr);
    h->rhs_cell = h->upload(cell);
    h->rhs_gidx = h->upload(gidx);
    h->rhs_coef = h->upload(coef);
}

// ---------------------------------------------------------------------------
// V-cycle (Algorithm 3)
template <typename T>
struct Prec;
template <>
struct Prec<double> {
    static double *u(DevLevel &D, int k) { return D.u64[k]; }
    static double *b(DevLevel &D) { return D.b64; }
    static double *rplg(DevLevel &D) { return D.rplg64; }
    static const double *fval(DevLevel &D) { return D.full_val64; }
    static PlgDev<double> &P(DevLevel &D) { return D.P64; }
};
template <>
struct Prec<float> {
    static float *u(DevLevel &D, int k) { return D.u32[k]; }
    static float *b(DevLevel &D) { return D.b32; }
    static float *rplg(DevLevel &D) { return D.rplg32; }
    static const float *fval(DevLevel &D) { return D.full_val32; }
    static PlgDev<float> &P(DevLevel &D) { return D.P32; }
};

// sweeps in pairs on this level in precision T (the tile lists are built
// for the tile height of the handle's cycle precision)
template <typename T>
bool use_pairs(const DevLevel &D) {
    return D.npair > 0 && (int)sizeof(T) == D.pair_word;
}

// one block-smoother sweep on level l (the iterate rotates through the
// level's buffers); uzero: the current iterate is known to be zero
template <typename T>
void smooth(mg_handle h, int l, bool uzero, hipStream_t st) {
    DevLevel &D = h->dev[l];
    const int nx = (D.cur + 1) % D.nbuf;
    T *uo = Prec<T>::u(D, D.cur), *un = Prec<T>::u(D, nx);
    // in timing mode: events around the finest level's tile kernel (levels
    // with two-sweep tiles time those instead)
    const bool rec = h->tim_capture && l == 0 && !use_pairs<T>(D) && 2 * h->ev_next + 1 < (int)h->ev.size();
    hipEvent_t e0 = rec ? h->ev[2 * h->ev_next] : nullptr, e1 = rec ? h->ev[2 * h->ev_next + 1] : nullptr;
    if (rec) ++h->ev_next;
    launch_smooth_a<T>(D.args, uo, Prec<T>::b(D), un, D.mask, uzero, Prec<T>::P(D), st, e0, e1);
    launch_smooth_b<T>(Prec<T>::P(D), un, st);
    D.cur = nx;
}

// n block-smoother sweeps on level l: in pairs where the level has two-sweep
// tiles, the last one alone when n is odd
template <typename T>
void smooth_n(mg_handle h, int l, int n, bool uzero, hipStream_t st) {
    DevLevel &D = h->dev[l];
    int k = 0;
    for (; use_pairs<T>(D) && k + 2 <= n; k += 2) {
        const int n1 = (D.cur + 1) % 3, n2 = (D.cur + 2) % 3;
        const bool rec = h->tim_capture && l == 0 && 2 * h->ev_next + 1 < (int)h->ev.size();
        hipEvent_t e0 = rec ? h->ev[2 * h->ev_next] : nullptr, e1 = rec ? h->ev[2 * h->ev_next + 1] : nullptr;
        if (rec) ++h->ev_next;
        launch_smooth_pair<T>(D.args, Prec<T>::u(D, D.cur), Prec<T>::b(D), Prec<T>::u(D, n1), Prec<T>::u(D, n2),
                              D.mask, uzero && k == 0, Prec<T>::P(D), D.pair_tiles, D.npair, D.single_tiles,
                              D.nsingle, st, e0, e1);
        D.cur = n2;
    }
    for (; k < n; ++k) smooth<T>(h, l, uzero && k == 0, st);
}

// Algorithm 3 on level l; uzero: the iterate on entry is zero (the coarse
// levels, and the FP32 cycle of the mixed-precision iteration)
template <typename T>
void vcycle(mg_handle h, int l, bool uzero, hipStream_t st) {
    DevLevel &D = h->dev[l];
    const int last = (int)h->dev.size() - 1;
    if (l == last) {
        launch_bottom<T, T>(D.nbot, D.bot_cells, D.ainv, Prec<T>::b(D), Prec<T>::u(D, D.cur), st);
        return;
    }
    const int nu1 = h->opt.nu1;
    if (nu1 == 0 && uzero) launch_fill_zero<T>(D.ncells, Prec<T>::u(D, D.cur), st);
    smooth_n<T>(h, l, nu1, uzero, st);
    DevLevel &C = h->dev[l + 1];
    T *u = Prec<T>::u(D, D.cur);
    // after a block-smoother sweep the PLG residuals are zero; without
    // pre-smoothing they are computed
    T *rplg = nullptr;
    if (nu1 == 0) {
        rplg = Prec<T>::rplg(D);
        launch_plg_residual<T>(D.m, D.plg_cell, D.full_ptr, D.full_col, Prec<T>::fval(D), Prec<T>::b(D), u, rplg, st);
    }
    C.cur = 0;
    launch_restrict<T>(D.args, C.args, u, Prec<T>::b(D), D.mask, D.plgidx, rplg, D.rmask, Prec<T>::b(C),
                       nu1 == 0 ? Prec<T>::u(C, 0) : nullptr, D.ex_nt, D.ex_ptr, D.ex_target, D.ex_child, true, st);
    vcycle<T>(h, l + 1, true, st);
    launch_prolong<T>(D.args, C.args, D.mask, C.mask, Prec<T>::u(C, C.cur), Prec<T>::u(D, D.cur), D.pex_n, D.pex_fine,
                      D.pex_coarse, false, st);
    smooth_n<T>(h, l, h->opt.nu2, false, st);
}

// Algorithm 4 on level l for the residual equation whose right-hand side is
// the level's b: restrict b down (eq. (5.8) on b itself), solve at the
// bottom, then on the way up start each level's V-cycle from the
// interpolated coarse result (eq. (5.9)).  The result is u(l, cur).
template <typename T>
void fmg(mg_handle h, int l, hipStream_t st) {
    DevLevel &D = h->dev[l];
    const int last = (int)h->dev.size() - 1;
    if (l == last) {
        launch_bottom<T, T>(D.nbot, D.bot_cells, D.ainv, Prec<T>::b(D), Prec<T>::u(D, D.cur), st);
        return;
    }
    DevLevel &C = h->dev[l + 1];
    launch_restrict<T>(D.args, C.args, nullptr, Prec<T>::b(D), D.mask, D.plgidx, nullptr, D.rmask, Prec<T>::b(C),
                       nullptr, D.ex_nt, D.ex_ptr, D.ex_target, D.ex_child, true, st);
    C.cur = 0;
    fmg<T>(h, l + 1, st);
    D.cur = 0;
    launch_prolong<T>(D.args, C.args, D.mask, C.mask, Prec<T>::u(C, C.cur), Prec<T>::u(D, 0), D.pex_n, D.pex_fine,
                      D.pex_coarse, true, st);
    vcycle<T>(h, l, false, st);
}

double device_absmax_finish(mg_handle h, int nblocks, hipStream_t st) {
    launch_absmax(nblocks, h->partial, nullptr, h->partial + h->npartial - 1, 1, st);
    HIPCHECK(hipMemcpyAsync(h->host_scalar, h->partial + h->npartial - 1, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    return *h->host_scalar;
}

double residual_norm(mg_handle h, int l, const double *u, const double *b, double *r64, hipStream_t st) {
    DevLevel &D = h->dev[l];
    int nb = launch_residual_norm(D.args, u, nullptr, false, nullptr, b, D.mask, D.m, D.plg_cell, D.fe_col, D.fe_val,
                                  nullptr, r64, h->partial, st);
    return device_absmax_finish(h, nb, st);
}

// Outer iterations either update u64[0] in place (FP64 V-cycles), or are
// in correction form (mixed precision, FMG): the cycle solves the residual
// equation from the residual left by the previous iteration, and the next
// residual pass adds its result e to u64[par], writing u64[1 - par].
bool correction_form(mg_handle h) { return h->opt.precision == MG_MIXED || h->opt.cycle == MG_CYCLE_FMG; }

// ||b - A u||_inf of the finest level into h->host_scalar[slot] (no
// synchronisation); u is u64[src] (+ e, written to u64[1 - src], when e is
// given); the residual itself goes to b32 (mixed) or r64 (FP64 FMG)
void enqueue_residual(mg_handle h, int src, const void *e, bool e64, int slot, hipStream_t st) {
    DevLevel &D = h->dev[0];
    const bool mixed = h->opt.precision == MG_MIXED;
    const bool fmg64 = !mixed && h->opt.cycle == MG_CYCLE_FMG;
    const int nb = launch_residual_norm(D.args, D.u64[src], e, e64, e ? D.u64[1 - src] : nullptr, D.b64, D.mask, D.m,
                                        D.plg_cell, D.fe_col, D.fe_val, mixed ? D.b32 : nullptr,
                                        fmg64 ? D.r64 : nullptr, h->partial, st);
    // the one-block reduction writes the norm straight into mapped host memory
    launch_absmax(nb, h->partial, nullptr, h->host_scalar_dev + slot, 1, st);
}

// one outer iteration on the handle's own buffers, then the residual
void enqueue_iteration(mg_handle h, int par, int slot, hipStream_t st) {
    DevLevel &D = h->dev[0];
    const bool mixed = h->opt.precision == MG_MIXED, fmg_cycle = h->opt.cycle == MG_CYCLE_FMG;
    D.cur = 0;
    if (mixed) {
        if (fmg_cycle) fmg<float>(h, 0, st);
        else vcycle<float>(h, 0, true, st);
        const float *e = D.u32[D.cur];
        D.cur = 0;
        enqueue_residual(h, par, e, false, slot, st);
    } else if (fmg_cycle) {
        // the FP64 cycle runs on the residual equation's own buffers
        std::swap(D.b64, D.r64);
        for (int k = 0; k < D.nbuf; ++k) std::swap(D.u64[k], D.e64[k]);
        fmg<double>(h, 0, st);
        const double *e = D.u64[D.cur];
        std::swap(D.b64, D.r64);
        for (int k = 0; k < D.nbuf; ++k) std::swap(D.u64[k], D.e64[k]);
        D.cur = 0;
        enqueue_residual(h, par, e, true, slot, st);
    } else {
        vcycle<double>(h, 0, false, st);
        if (D.cur != 0) HIPCHECK(hipMemcpyAsync(D.u64[0], D.u64[D.cur], D.ncells * 8, hipMemcpyDeviceToDevice, st));
        D.cur = 0;
        enqueue_residual(h, 0, nullptr, false, slot, st);
    }
}

// k outer iterations (k = 1, 2, 4 or 8); residual norms in
// h->host_scalar[0, k)
void run_iterations(mg_handle h, int k, hipStream_t st) {
    const bool corr = correction_form(h);
    const int par = corr ? h->upar : 0;
    const int p = corr ? 1 + par : 0, c = k == 1 ? 0 : k == 2 ? 1 : k == 4 ? 2 : 3;
    auto enqueue = [&](hipStream_t s) {
        for (int i = 0; i < k; ++i) enqueue_iteration(h, corr ? (par + i) & 1 : 0, i, s);
    };
    if (h->eager || h->timing) {
        // kernel timing: eager launches, an event pair taking the start and
        // end of each finest-level tile kernel (HIP events recorded inside
        // graphs cannot be timed)
        h->ev_next = 0;
        h->tim_capture = h->timing;
        enqueue(st);
        h->tim_capture = false;
        h->tim_last = h->timing ? h->ev_next : 0;
        if (corr && (k & 1)) h->upar = 1 - h->upar;
        return;
    }
    if (!h->iter_exec[p][c]) {
        std::lock_guard<std::mutex> lk(g_capture_mu);
        if (!h->cap_stream) HIPCHECK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
        HIPCHECK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
        enqueue(h->cap_stream);
        HIPCHECK(hipStreamEndCapture(h->cap_stream, &h->iter_graph[p][c]));
        HIPCHECK(hipGraphInstantiate(&h->iter_exec[p][c], h->iter_graph[p][c], nullptr, nullptr, 0));
    }
    HIPCHECK(hipGraphLaunch(h->iter_exec[p][c], st));
    if (corr && (k & 1)) h->upar = 1 - h->upar;
}

// after the stream has been synchronised: add the durations recorded by the
// last timing replay
void collect_timing(mg_handle h) {
    for (int q = 0; q < h->tim_last; ++q) {
        float ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, h->ev[2 * q], h->ev[2 * q + 1]));
        h->tim_total_ms += ms;
        ++h->nrec;
    }
    h->tim_last = 0;
}

thread_local std::string g_last_error;

mg_status guard(mg_handle h, const std::function<void()> &fn) {
    try {
        fn();
        return MG_OK;
    } catch (const status_error &e) {
        g_last_error = e.what();
        if (h) h->last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return MG_ERR_OOM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        if (h) h->last_error = e.what();
        return MG_ERR_INVALID_ARG;
    }
}

// Nodes and weights (divided by the cell volume) of the cut-cell quadrature:
// cell(c0, first) is called before the nodes of each active irregular cell,
// node(x, y, w) for every node.
template <typename CellFn, typename NodeFn>
void cut_cell_nodes(mg_handle h, CellFn cell, NodeFn node) {
    const Level &L = *h->levels[0];
    const CutGrid &cg = L.cg;
    std::vector<double> g16x, g16w, g8x, g8w;
    gauss_legendre(16, g16x, g16w);
    gauss_legendre(8, g8x, g8w);
    const double hh = L.g.h;
    for (size_t s = 0; s < cg.irr_cells.size(); ++s) {
        const int c0 = cg.irr_cells[s];
        const CellData &d = cg.irr[s];
        if (!cg.active[c0]) continue;
        const double vol = d.mom[0] * hh * hh;
        cell(c0, true);
        auto emit = [&](double px, double py, double pw) { node(px, py, pw / vol); };
        for (int ci : d.members) {
            const Comp &c = cg.comps[ci];
            const double X0 = L.g.x0 + c.ci * hh, Y0 = L.g.y0 + c.cj * hh, xr = X0 + 0.5 * hh;
            if (c.full) {
                for (int a = 0; a < 8; ++a)
                    for (int b = 0; b < 8; ++b)
                        emit(X0 + (0.5 + 0.5 * g8x[a]) * hh, Y0 + (0.5 + 0.5 * g8x[b]) * hh, 0.25 * hh * hh * g8w[a] * g8w[b]);
                continue;
            }
            for (const LoopItem &it : c.items) {
                if (!it.is_edge) {
                    const Seg &sg = h->curves.c[it.piece.curve][it.piece.seg];
                    for (int k = 0; k < 16; ++k) {
                        double t = 0.5 * (it.piece.tb - it.piece.ta) * g16x[k] + 0.5 * (it.piece.ta + it.piece.tb);
                        double px, py, dx, dy;
                        sg.point(t, px, py);
                        sg.deriv(t, dx, dy);
                        double ow = 0.5 * (it.piece.tb - it.piece.ta) * g16w[k] * dy;
                        double half = 0.5 * (px - xr);
                        for (int q = 0; q < 16; ++q) emit(xr + half * (1.0 + g16x[q]), py, ow * g16w[q] * half);
                    }
                } else if (it.side == 1 || it.side == 3) {
                    double px = it.side == 1 ? X0 + hh : X0;
                    double ya = it.side == 1 ? Y0 + it.s0 * hh : Y0 + (1.0 - it.s0) * hh;
                    double yb = it.side == 1 ? Y0 + it.s1 * hh : Y0 + (1.0 - it.s1) * hh;
                    for (int k = 0; k < 8; ++k) {
                        double py = 0.5 * (yb - ya) * g8x[k] + 0.5 * (ya + yb);
                        double ow = 0.5 * (yb - ya) * g8w[k];
                        double half = 0.5 * (px - xr);
                        for (int q = 0; q < 16; ++q) emit(xr + half * (1.0 + g16x[q]), py, ow * g16w[q] * half);
                    }
                }
            }
        }
    }
}

// Nodes of the boundary data in the layout of g: entry() before each entry
// (box faces bottom, top, left, right, then irregular cells), node(x, y, w,
// nx, ny, curve, seg) with weights summing to 1 per entry and the outward
// unit normal.
template <typename EntryFn, typename NodeFn>
void boundary_nodes(mg_handle h, EntryFn entry, NodeFn node) {
    const Level &L = *h->levels[0];
    const CutGrid &cg = L.cg;
    const int nx = L.g.nx, ny = L.g.ny;
    const double hh = L.g.h;
    std::vector<double> g16x, g16w, g8x, g8w;
    gauss_legendre(16, g16x, g16w);
    gauss_legendre(8, g8x, g8w);
    const double x1 = L.g.x0 + nx * hh, y1 = L.g.y0 + ny * hh;
    for (int side : {0, 2, 3, 1}) {
        const int m = (side == 0 || side == 2) ? nx : ny;
        for (int k = 0; k < m; ++k) {
            entry();
            for (int q = 0; q < 8; ++q) {
                double s = L.g.x0 + (k + 0.5 + 0.5 * g8x[q]) * hh, tt = L.g.y0 + (k + 0.5 + 0.5 * g8x[q]) * hh;
                if (side == 0) node(s, L.g.y0, 0.5 * g8w[q], 0.0, -1.0, 0, side);
                else if (side == 2) node(s, y1, 0.5 * g8w[q], 0.0, 1.0, 0, side);
                else if (side == 3) node(L.g.x0, tt, 0.5 * g8w[q], -1.0, 0.0, 0, side);
                else node(x1, tt, 0.5 * g8w[q], 1.0, 0.0, 0, side);
            }
        }
    }
    for (int cl = 0; cl < nx * ny; ++cl) {
        if (L.g_of_cell[cl] < 0) continue;
        const CellData &d = cg.irr[cg.irr_slot[cl]];
        entry();
        double len = 0.0;
        for (auto &bp : d.bp) {
            const Seg &sg = h->curves.c[bp.curve][bp.seg];
            for (int q = 0; q < 16; ++q) {
                double t = 0.5 * (bp.tb - bp.ta) * g16x[q] + 0.5 * (bp.ta + bp.tb), dx, dy;
                sg.deriv(t, dx, dy);
                len += 0.5 * (bp.tb - bp.ta) * g16w[q] * std::hypot(dx, dy);
            }
        }
        for (auto &bp : d.bp) {
            const Seg &sg = h->curves.c[bp.curve][bp.seg];
            for (int q = 0; q < 16; ++q) {
                double t = 0.5 * (bp.tb - bp.ta) * g16x[q] + 0.5 * (bp.ta + bp.tb), px, py, dx, dy;
                sg.point(t, px, py);
                sg.deriv(t, dx, dy);
                double sp = std::hypot(dx, dy);
                node(px, py, 0.5 * (bp.tb - bp.ta) * g16w[q] * sp / len, dy / sp, -dx / sp, bp.curve, bp.seg);
            }
        }
    }
}

// b_{l+1} = R (b - A u) on level l with every residual computed (also on PLG rows)
template <typename T>
void restrict_step(mg_handle h, int level, const T *b, const T *u, T *bc, hipStream_t st) {
    DevLevel &D = h->dev[level], &C = h->dev[level + 1];
    T *rplg = Prec<T>::rplg(D);
    launch_plg_residual<T>(D.m, D.plg_cell, D.full_ptr, D.full_col, Prec<T>::fval(D), b, u, rplg, st);
    launch_restrict<T>(D.args, C.args, u, b, D.mask, D.plgidx, rplg, D.rmask, bc, nullptr, D.ex_nt, D.ex_ptr,
                       D.ex_target, D.ex_child, false, st);
}

}  // namespace

// ===========================================================================
extern "C" {

mg_status mg_default_options(mg_options *opt) {
    if (!opt) return MG_ERR_INVALID_ARG;
    opt->eps = 0.08;
    opt->omega = 0.5;
    opt->nu1 = 3;
    opt->nu2 = 3;
    opt->n_levels = 0;
    opt->min_coarse = 16;
    opt->precision = MG_FP64;
    opt->max_iters = 100;
    opt->cycle = MG_CYCLE_V;
    opt->degree = 4;
    opt->w_min = 0.5;
    opt->colouring = MG_SMOOTH_JACOBI;
    opt->split_cells = 0;
    opt->small_cells = 0;
    opt->split_b_sep = 0;
    opt->seg_max = 0;
    opt->seg_whole = 0;
    opt->pair_sweeps = 0;
    return MG_OK;
}

mg_status mg_setup(const mg_grid *grid, int n_curves, const mg_curve *curves, double a, double b, double c,
                   const mg_options *opt, void *stream, mg_handle *out) {
    if (!grid || !curves || !out || n_curves < 1) return MG_ERR_INVALID_ARG;
    *out = nullptr;
    if (!(b * b - 4 * a * c < 0) || !(a > 0 || a < 0) || std::isnan(a) || std::isnan(b) || std::isnan(c))
        return MG_ERR_INVALID_ARG;
    if (grid->nx < 4 || grid->ny < 4 || !(grid->h > 0) || (long long)grid->nx * grid->ny > (1LL << 28))
        return MG_ERR_INVALID_ARG;
    mg_options o;
    mg_default_options(&o);
    if (opt) o = *opt;
    if (!(o.eps > 0 && o.eps < 1) || o.nu1 < 0 || o.nu2 < 0 || o.max_iters < 1 || o.min_coarse < 4 ||
        (o.precision != MG_FP64 && o.precision != MG_MIXED) || o.n_levels < 0 || o.n_levels > 16 ||
        (o.cycle != MG_CYCLE_V && o.cycle != MG_CYCLE_FMG) || !(o.omega > 0 && o.omega < 2) ||
        !(o.w_min > 0 && o.w_min < 1e6) || (o.colouring != MG_SMOOTH_JACOBI && o.colouring != MG_SMOOTH_MULTICOLOUR) ||
        o.split_cells < 0 || o.small_cells < -1 || o.split_b_sep < 0 || o.seg_max < 0 ||
        (o.seg_max > 0 && (o.seg_max < 32 || o.seg_max > PLG_LMAX)) || o.seg_whole < 0 || o.seg_whole > PLG_LMAX ||
        (o.pair_sweeps != 0 && o.pair_sweeps != -1))
        return MG_ERR_INVALID_ARG;
    if (o.degree != 4) {
        g_last_error = "only degree-4 fits (lattices of 15 cells) are built";
        return MG_ERR_UNSUPPORTED;
    }
    for (int k = 0; k < n_curves; ++k) {
        if (curves[k].n_seg < 1 || !curves[k].seg) return MG_ERR_INVALID_ARG;
        for (int s = 0; s < curves[k].n_seg; ++s) {
            const mg_segment &sg = curves[k].seg[s];
            if ((sg.kind != MG_SEG_LINE && sg.kind != MG_SEG_ARC && sg.kind != MG_SEG_CUBIC) || sg.bc < 0 ||
                sg.bc > 3)
                return MG_ERR_INVALID_ARG;
            const int np = sg.kind == MG_SEG_LINE ? 4 : sg.kind == MG_SEG_ARC ? 5 : 8;
            for (int t = 0; t < np; ++t)
                if (!std::isfinite(sg.p[t])) return MG_ERR_INVALID_ARG;
        }
    }
    auto h = std::make_unique<mg_handle_s>();
    hipStream_t st = (hipStream_t)stream;
    mg_status rc = guard(h.get(), [&]() {
        // the host-side geometry, lattice and solver work runs without the
        // capture lock; device allocations, copies and the fits take it
        auto t0 = std::chrono::steady_clock::now();
        HIPCHECK(hipGetDevice(&h->device));
        h->scratch = noalloc_scratch();
        if (!h->scratch) fail(MG_ERR_HIP, "hipGetSymbolAddress of the fixed scratch failed");
        h->opt = o;
        h->a = a; h->b = b; h->c = c;
        for (int k = 0; k < n_curves; ++k) {
            std::vector<Seg> segs;
            for (int s = 0; s < curves[k].n_seg; ++s) {
                const mg_segment &sg = curves[k].seg[s];
                Seg q;
                q.kind = sg.kind;
                for (int t = 0; t < 8; ++t) q.p[t] = sg.kind == MG_SEG_CUBIC || t < 5 ? sg.p[t] : 0.0;
                q.bc = sg.bc;
                q.al1 = sg.alpha1;
                q.al2 = sg.alpha2;
                segs.push_back(q);
            }
            h->curves.c.push_back(segs);
        }
        mg_grid g = *grid;
        while (true) {
            auto L = std::make_unique<Level>();
            L->g = g;
            L->a = a; L->b = b; L->c = c;
            L->curves = &h->curves;
            L->w_min = o.w_min;
            try {
                auto c0 = std::chrono::steady_clock::now();
                build_cutgrid(h->curves, g, o.eps, L->cg);
                auto c1 = std::chrono::steady_clock::now();
                h->stage[0] += std::chrono::duration<double>(c1 - c0).count();
                L->classify();
                h->stage[1] += std::chrono::duration<double>(std::chrono::steady_clock::now() - c1).count();
                fit_level(h.get(), *L, st);
            } catch (const status_error &e) {
                if (h->levels.empty() || e.code != MG_ERR_GEOMETRY || o.n_levels) throw;
                break;
            }
            h->levels.push_back(std::move(L));
            if (o.n_levels && (int)h->levels.size() == o.n_levels) break;
            if (g.nx % 2 || g.ny % 2 || g.nx / 2 < o.min_coarse || g.ny / 2 < o.min_coarse) {
                if (o.n_levels) fail(MG_ERR_GEOMETRY, "cannot build the requested number of levels");
                break;
            }
            if (h->levels.size() == 16) break;
            g.h *= 2;
            g.nx /= 2;
            g.ny /= 2;
        }
        const int nl = (int)h->levels.size();
        auto s0 = std::chrono::steady_clock::now();
        h->solvers.resize(nl);
        h->cond_a22.assign(nl, 0.0);
        for (int l = 0; l < nl; ++l) {
            // whole chains as segments when that leaves no separators (one
            // smoother launch per sweep), else short segments
            build_plg_solver(*h->levels[l], o.seg_whole > 0 ? o.seg_whole : SEG_WHOLE, h->solvers[l]);
            if (h->solvers[l].nsep > 0)
                build_plg_solver(*h->levels[l], o.seg_max > 0 ? o.seg_max : SEG_MAX, h->solvers[l]);
            h->cond_a22[l] = cond1_estimate(*h->levels[l], h->solvers[l]);
        }
        h->stage[3] += std::chrono::duration<double>(std::chrono::steady_clock::now() - s0).count();
        std::lock_guard<std::mutex> lk(g_capture_mu);
        h->dev.resize(nl);
        for (int l = 0; l < nl; ++l) upload_level(h.get(), l, l == nl - 1, st);
        upload_rhs(h.get());
        if (o.cycle == MG_CYCLE_FMG && o.precision == MG_FP64) {
            DevLevel &D0 = h->dev[0];
            D0.r64 = h->alloc<double>(D0.ncells);
            for (int k = 0; k < D0.nbuf; ++k) D0.e64[k] = h->alloc<double>(D0.ncells);
        }
        int maxblk = 1;
        for (auto &D : h->dev)
            maxblk = std::max(maxblk, ((D.args.nx + 63) / 64) * ((D.args.ny + 31) / 32) + (D.m + 255) / 256);
        h->npartial = std::max(maxblk, 1024) + 1;
        h->partial = h->alloc<double>(h->npartial);
        HIPCHECK(hipHostMalloc((void **)&h->host_scalar, sizeof(double) * ITER_CHUNK,
                               hipHostMallocMapped | hipHostMallocCoherent));
        HIPCHECK(hipHostGetDevicePointer((void **)&h->host_scalar_dev, h->host_scalar, 0));
        HIPCHECK(hipStreamSynchronize(st));
        h->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        h->stage[5] = std::max(0.0, h->setup_seconds - (h->stage[0] + h->stage[1] + h->stage[2] + h->stage[3] +
                                                        h->stage[4]));
    });
    if (rc != MG_OK) {
        mg_destroy(h.release());
        return rc;
    }
    *out = h.release();
    return MG_OK;
}

mg_status mg_rhs(mg_handle h, const double *f_dev, const double *g_dev, double *b_dev, void *stream) {
    if (!h || !f_dev || !b_dev || (!g_dev && h->nrhs)) return MG_ERR_INVALID_ARG;
    return guard(h, [&]() {
        DevLevel &D = h->dev[0];
        launch_rhs(D.ncells, D.mask, f_dev, b_dev, h->nrhs, h->rhs_ptr, h->rhs_cell, h->rhs_gidx, h->rhs_coef, g_dev,
                   (hipStream_t)stream);
        HIPCHECK(hipGetLastError());
    });
}

mg_status mg_vcycle(mg_handle h, const double *b_dev, double *u_dev, void *stream) {
    if (!h || !b_dev || !u_dev) return MG_ERR_INVALID_ARG;
    return guard(h, [&]() {
        hipStream_t st = (hipStream_t)stream;
        DevLevel &D = h->dev[0];
        double *keep_u = D.u64[0], *keep_b = D.b64;
        D.u64[0] = u_dev;
        D.b64 = const_cast<double *>(b_dev);
        D.cur = 0;
        vcycle<double>(h, 0, false, st);
        if (D.cur != 0) HIPCHECK(hipMemcpyAsync(u_dev, D.u64[D.cur], D.ncells * 8, hipMemcpyDeviceToDevice, st));
        D.u64[0] = keep_u;
        D.b64 = keep_b;
        D.cur = 0;
        HIPCHECK(hipGetLastError());
    });
}

mg_status mg_smooth(mg_handle h, int level, const double *b_dev, double *u_dev, void *stream) {
    if (!h || !b_dev || !u_dev || level < 0 || level >= (int)h->dev.size()) return MG_ERR_INVALID_ARG;
    return guard(h, [&]() {
        hipStream_t st = (hipStream_t)stream;
        DevLevel &D = h->dev[level];
        launch_smooth_a<double>(D.args, u_dev, b_dev, D.u64[1], D.mask, false, D.P64, st);
        launch_smooth_b<double>(D.P64, D.u64[1], st);
        HIPCHECK(hipMemcpyAsync(u_dev, D.u64[1], D.ncells * 8, hipMemcpyDeviceToDevice, st));
        HIPCHECK(hipGetLastError());
    });
}

mg_status mg_smooth32(mg_handle h, int level, const float *b_dev, float *u_dev, void *stream) {
    if (!h || !b_dev || !u_dev || level < 0 || level >= (int)h->dev.size()) return MG_ERR_INVALID_ARG;
    return guard(h, [&]() {
        hipStream_t st = (hipStream_t)stream;
        DevLevel &D = h->dev[level];
        launch_smooth_a<float>(D.args, u_dev, b_dev, D.u32[1], D.mask, false, D.P32, st);
        launch_smooth_b<float>(D.P32, D.u32[1], st);
        HIPCHECK(hipMemcpyAsync(u_dev, D.u32[1], D.ncells * 4, hipMemcpyDeviceToDevice, st));
        HIPCHECK(hipGetLastError());
    });
}

mg_status mg_restrict(mg_handle h, int level, int precision, const void *b_dev, const void *u_dev, void *bc_dev,
                      void *stream) {
    if (!h || !b_dev || !u_dev || !bc_dev || level < 0 || level + 1 >= (int)h->dev.size() ||
        (precision != MG_FP64 && precision != MG_MIXED))
        return MG_ERR_INVALID_ARG;
    return guard(h, [&]() {
        hipStream_t st = (hipStream_t)stream;
        if (precision == MG_FP64)
            restrict_step<double>(h, level, (const double *)b_dev, (const double *)u_dev, (double *)bc_dev, st);
        else
            restrict_step<float>(h, level, (const float *)b_dev, (const float *)u_dev, (float *)bc_dev, st);
        HIPCHECK(hipGetLastError());
    });
}

mg_status mg_prolong(mg_handle h, int level, int precision, const void *ec_dev, void *u_dev, void *stream) {
    if (!h || !ec_dev || !u_dev || level < 0 || level + 1 >= (int)h->dev.size() ||
        (precision != MG_FP64 && precision != MG_MIXED))
        return MG_ERR_INVALID_ARG;
    return guard(h, [&]() {
        hipStream_t st = (hipStream_t)stream;
        DevLevel &D = h->dev[level], &C = h->dev[level + 1];
        if (precision == MG_FP64)
            launch_prolong<double>(D.args, C.args, D.mask, C.mask, (const double *)ec_dev, (double *)u_dev, D.pex_n,
                                   D.pex_fine, D.pex_coarse, false, st);
        else
            launch_prolong<float>(D.args, C.args, D.mask, C.mask, (const float *)ec_dev, (float *)u_dev, D.pex_n,
                                  D.pex_fine, D.pex_coarse, false, st);
        HIPCHECK(hipGetLastError());
    });
}

mg_status mg_residual(mg_handle h, int level, const double *b_dev, const double *u_dev, double *r_dev, double *rnorm,
                      void *stream) {
    if (!h || !b_dev || !u_dev || level < 0 || level >= (int)h->dev.size()) return MG_ERR_INVALID_ARG;
    return guard(h, [&]() {
        double v = residual_norm(h, level, u_dev, b_dev, r_dev, (hipStream_t)stream);
        if (rnorm) *rnorm = v;
    });
}

mg_status mg_residual_norm_noalloc(mg_handle h, int level, const double *b_dev, const double *u_dev, double *r_dev,
                                   double *rnorm_dev, void *stream) {
    if (!h || !b_dev || !u_dev || !rnorm_dev || level < 0 || level >= (int)h->dev.size()) return MG_ERR_INVALID_ARG;
    DevLevel &D = h->dev[level];
    const int nb = residual_norm_blocks(D.args, D.m);
    if (nb > NOALLOC_SCRATCH_DOUBLES) {
        g_last_error = "mg_residual_norm_noalloc: the level needs " + std::to_string(nb) +
                       " partial maxima, more than the fixed scratch holds (" +
                       std::to_string(NOALLOC_SCRATCH_DOUBLES) + ")";
        return MG_ERR_UNSUPPORTED;
    }
    if (!h->scratch) return MG_ERR_HIP;
    return guard(h, [&]() {
        hipStream_t st = (hipStream_t)stream;
        const int n = launch_residual_norm(D.args, u_dev, nullptr, false, nullptr, b_dev, D.mask, D.m, D.plg_cell,
                                           D.fe_col, D.fe_val, nullptr, r_dev, h->scratch, st);
        launch_absmax(n, h->scratch, nullptr, rnorm_dev, 1, st);
        HIPCHECK(hipGetLastError());
    });
}

mg_status mg_solve(mg_handle h, const double *f_dev, const double *g_dev, double *u_dev, double tol, void *stream,
                   int *iters, double *rel_residual) {
    if (!h || !f_dev || !u_dev || !(tol > 0) || (!g_dev && h->nrhs)) return MG_ERR_INVALID_ARG;
    mg_status result = MG_OK;
    mg_status rc = guard(h, [&]() {
        hipStream_t st = (hipStream_t)stream;
        DevLevel &D = h->dev[0];
        launch_rhs(D.ncells, D.mask, f_dev, D.b64, h->nrhs, h->rhs_ptr, h->rhs_cell, h->rhs_gidx, h->rhs_coef, g_dev, st);
        int nb = 1024;
        launch_absmax((int)D.ncells, D.b64, D.mask, h->partial, nb, st);
        double bnorm = device_absmax_finish(h, nb, st);
        if (bnorm == 0.0) bnorm = 1.0;
        const bool mixed = h->opt.precision == MG_MIXED;
        // iterate on the handle's own finest-level buffer (fixed addresses,
        // so the captured iteration can be replayed)
        HIPCHECK(hipMemcpyAsync(D.u64[0], u_dev, D.ncells * 8, hipMemcpyDeviceToDevice, st));
        h->upar = 0;
        enqueue_residual(h, 0, nullptr, false, 0, st);
        HIPCHECK(hipStreamSynchronize(st));
        int it = 0, grow = 0;
        double rel = h->host_scalar[0] / bnorm;
        double prev = rel, rmin = 1.0;
        int nratio = 0;
        bool stop = false;
        while (!stop && rel > tol && it < h->opt.max_iters) {
            // several iterations per launch (one host round trip) while the
            // tolerance cannot be reached within them even at 1.5 times the
            // fastest logarithmic rate seen so far
            int k = 1;
            if (nratio >= 2 && rmin > 0.0 && rmin < 1.0) {
                const double need = std::log(tol / rel) / (1.5 * std::log(rmin));
                while (k < ITER_CHUNK && need >= 2 * k + 1 && it + 2 * k <= h->opt.max_iters) k *= 2;
            }
            run_iterations(h, k, st);
            HIPCHECK(hipStreamSynchronize(st));
            if (h->timing) collect_timing(h);
            for (int i = 0; i < k && !stop; ++i) {
                ++it;
                rel = h->host_scalar[i] / bnorm;
                if (std::isnan(rel)) { result = MG_ERR_DIVERGED; stop = true; break; }
                grow = rel > prev ? grow + 1 : 0;
                if (grow >= 3) { result = MG_ERR_DIVERGED; stop = true; break; }
                if (prev > 0.0) {
                    const double q = rel / prev;
                    rmin = nratio == 0 ? q : std::min(rmin, q);
                    ++nratio;
                }
                prev = rel;
            }
        }
        HIPCHECK(hipMemcpyAsync(u_dev, D.u64[correction_form(h) ? h->upar : 0], D.ncells * 8,
                                hipMemcpyDeviceToDevice, st));
        launch_zero_inactive(D.ncells, D.mask, u_dev, st);
        HIPCHECK(hipStreamSynchronize(st));
        if (result == MG_OK && rel > tol) result = MG_ERR_NO_CONVERGENCE;
        if (iters) *iters = it;
        if (rel_residual) *rel_residual = rel;
    });
    return rc != MG_OK ? rc : result;
}

mg_status mg_query(mg_handle h, mg_info *info) {
    if (!h || !info) return MG_ERR_INVALID_ARG;
    std::memset(info, 0, sizeof(*info));
    info->n_levels = (int)h->levels.size();
    for (int l = 0; l < info->n_levels && l < 16; ++l) {
        const Level &L = *h->levels[l];
        info->nx[l] = L.g.nx;
        info->ny[l] = L.g.ny;
        info->n_active[l] = L.n_active;
        info->n_plg[l] = (int)L.plg_cells.size();
        info->n_sep[l] = h->solvers[l].nsep;
        info->sweep_words[l] = h->dev[l].sweep_words;
        info->n_sfv[l] = h->dev[l].nsfv;
        info->cond_A22[l] = l < (int)h->cond_a22.size() ? h->cond_a22[l] : 0.0;
        info->n_pair_sfv[l] = h->dev[l].n_pair_sfv;
        info->nnz_plg += (long long)L.col.size();
    }
    info->n_face = h->levels[0]->n_face;
    info->n_irr = h->levels[0]->n_irr;
    info->device_bytes = h->bytes;
    info->setup_seconds = h->setup_seconds;
    for (int k = 0; k < 6; ++k) info->setup_stage_seconds[k] = h->stage[k];
    return MG_OK;
}

mg_status mg_export_level(mg_handle h, int level, int *kind, int *n_plg, long long *nnz, int *row_ptr, int *col,
                          double *val, double *beta_b) {
    if (!h || level < 0 || level >= (int)h->levels.size()) return MG_ERR_INVALID_ARG;
    const Level &L = *h->levels[level];
    if (kind) for (size_t k = 0; k < L.kind.size(); ++k) kind[k] = L.kind[k];
    if (n_plg) *n_plg = (int)L.plg_cells.size();
    if (nnz) *nnz = (long long)L.col.size();
    if (col) {
        if (!row_ptr || !val) return MG_ERR_INVALID_ARG;
        for (size_t k = 0; k < L.row_ptr.size(); ++k) row_ptr[k] = L.row_ptr[k];
        for (size_t k = 0; k < L.col.size(); ++k) {
            col[k] = L.col[k];
            val[k] = L.val[k];
        }
        if (beta_b) for (size_t k = 0; k < L.beta_b.size(); ++k) beta_b[k] = L.beta_b[k];
    }
    return MG_OK;
}

// Quadrature for cell averages over irregular cells: Green's theorem,
// ∬ F = ∮ G dy with G(x, y) the integral of F(., y) from the cell-centre
// abscissa to x; Gauss-Legendre along each boundary piece (16 points on curve
// pieces, 8 on cell sides) times 16 inner points; full grid cells absorbed by
// a merge use an 8 x 8 tensor rule.  Weights are divided by the cell volume.
mg_status mg_cell_quadrature(mg_handle h, int *n, long long *nnodes, int *cell, long long *ptr, double *x, double *y,
                             double *w) {
    if (!h || !n || !nnodes) return MG_ERR_INVALID_ARG;
    long long cnt = 0;
    int ncell = 0;
    cut_cell_nodes(h, [&](int c0, bool first) {
        if (first) {
            if (ptr && x) ptr[ncell] = cnt;
            if (cell && x) cell[ncell] = c0;
            ++ncell;
        }
    }, [&](double px, double py, double pw) {
        if (x) {
            x[cnt] = px;
            y[cnt] = py;
            w[cnt] = pw;
        }
        ++cnt;
    });
    if (ptr && x) ptr[ncell] = cnt;
    *n = ncell;
    *nnodes = cnt;
    return MG_OK;
}

// Quadrature for the boundary data g: 8 Gauss points per box face, 16 per
// curve piece of an irregular cell, weights normalised to 1 per entry.
mg_status mg_boundary_quadrature(mg_handle h, int *n, long long *nnodes, long long *ptr, double *x, double *y,
                                 double *w, double *nxo, double *nyo, int *bc, double *alpha1, double *alpha2) {
    if (!h || !n || !nnodes) return MG_ERR_INVALID_ARG;
    long long cnt = 0;
    int entry = 0;
    boundary_nodes(h, [&]() {
        if (ptr && x) ptr[entry] = cnt;
        ++entry;
    }, [&](double px, double py, double pw, double n0, double n1, int curve, int seg) {
        if (x) {
            const Seg &sg = h->curves.c[curve][seg];
            x[cnt] = px; y[cnt] = py; w[cnt] = pw; nxo[cnt] = n0; nyo[cnt] = n1;
            bc[cnt] = sg.bc; alpha1[cnt] = sg.al1; alpha2[cnt] = sg.al2;
        }
        ++cnt;
    });
    if (ptr && x) ptr[entry] = cnt;
    *n = entry;
    *nnodes = cnt;
    return MG_OK;
}

mg_status mg_project_rhs(mg_handle h, mg_f_batch f, mg_g_batch g, void *ctx, int gauss_points, double *f_dev,
                         double *g_dev, void *stream) {
    if (!h || !f || !f_dev || gauss_points < 1 || gauss_points > 16) return MG_ERR_INVALID_ARG;
    if (h->levels[0]->n_face + h->levels[0]->n_irr > 0 && (!g || !g_dev)) return MG_ERR_INVALID_ARG;
    return guard(h, [&]() {
        const Level &L = *h->levels[0];
        const int nx = L.g.nx, ny = L.g.ny;
        const double hh = L.g.h;
        const size_t pitch = (size_t)nx + 4;
        std::vector<double> fh((size_t)(ny + 4) * pitch, 0.0);
        constexpr long long CHUNK = 1 << 20;
        std::vector<double> bx, by, bw, bo;
        std::vector<long long> dst;        // padded cell (f) or entry (g) per node
        std::vector<int> bcv, bsg;
        std::vector<double> bnx, bny;
        // f: tensor Gauss-Legendre on full cells, the library's cut-cell rule
        // on the others
        auto flush_f = [&]() {
            if (bx.empty()) return;
            bo.assign(bx.size(), 0.0);
            f((long long)bx.size(), bx.data(), by.data(), bo.data(), ctx);
            for (size_t k = 0; k < bx.size(); ++k) fh[dst[k]] += bw[k] * bo[k];
            bx.clear(); by.clear(); bw.clear(); dst.clear();
        };
        std::vector<double> gx, gw;
        gauss_legendre(gauss_points, gx, gw);
        std::vector<char> cut((size_t)nx * ny, 0);
        for (size_t s = 0; s < L.cg.irr_cells.size(); ++s) cut[L.cg.irr_cells[s]] = 1;
        for (int cl = 0; cl < nx * ny; ++cl) {
            if (!L.cg.active[cl] || cut[cl]) continue;
            const double X0 = L.g.x0 + (cl % nx) * hh, Y0 = L.g.y0 + (cl / nx) * hh;
            const long long pc = (long long)padded_index(nx, cl);
            for (int a = 0; a < gauss_points; ++a)
                for (int b = 0; b < gauss_points; ++b) {
                    bx.push_back(X0 + (0.5 + 0.5 * gx[a]) * hh);
                    by.push_back(Y0 + (0.5 + 0.5 * gx[b]) * hh);
                    bw.push_back(0.25 * gw[a] * gw[b]);
                    dst.push_back(pc);
                }
            if ((long long)bx.size() >= CHUNK) flush_f();
        }
        long long cur_cell = 0;
        cut_cell_nodes(h, [&](int c0, bool first) {
            if (first) cur_cell = (long long)padded_index(nx, c0);
        }, [&](double px, double py, double pw) {
            bx.push_back(px);
            by.push_back(py);
            bw.push_back(pw);
            dst.push_back(cur_cell);
            if ((long long)bx.size() >= CHUNK) flush_f();
        });
        flush_f();
        // g: boundary averages of the data in the library's layout
        const int nent = L.n_face + L.n_irr;
        std::vector<double> gh(std::max(nent, 1), 0.0);
        auto flush_g = [&]() {
            if (bx.empty()) return;
            bo.assign(bx.size(), 0.0);
            g((long long)bx.size(), bx.data(), by.data(), bcv.data(), bsg.data(), bnx.data(), bny.data(), bo.data(),
              ctx);
            for (size_t k = 0; k < bx.size(); ++k) gh[dst[k]] += bw[k] * bo[k];
            bx.clear(); by.clear(); bw.clear(); dst.clear(); bcv.clear(); bsg.clear(); bnx.clear(); bny.clear();
        };
        long long entry = -1;
        if (g) {
            boundary_nodes(h, [&]() { ++entry; }, [&](double px, double py, double pw, double n0, double n1, int curve,
                                                     int seg) {
                bx.push_back(px); by.push_back(py); bw.push_back(pw); dst.push_back(entry);
                bcv.push_back(curve); bsg.push_back(seg); bnx.push_back(n0); bny.push_back(n1);
                if ((long long)bx.size() >= CHUNK) flush_g();
            });
            flush_g();
        }
        hipStream_t st = (hipStream_t)stream;
        HIPCHECK(hipMemcpyAsync(f_dev, fh.data(), fh.size() * 8, hipMemcpyHostToDevice, st));
        if (g && nent > 0) HIPCHECK(hipMemcpyAsync(g_dev, gh.data(), (size_t)nent * 8, hipMemcpyHostToDevice, st));
        HIPCHECK(hipStreamSynchronize(st));
    });
}

mg_status mg_kernel_timing(mg_handle h, int enable, int *launches, double *avg_ms) {
    if (!h) return MG_ERR_INVALID_ARG;
    return guard(h, [&]() {
        if (enable) {
            const int pairs = ITER_CHUNK * std::max(1, h->opt.nu1 + h->opt.nu2);
            if ((int)h->ev.size() < 2 * pairs) {
                std::lock_guard<std::mutex> lk(g_capture_mu);
                while ((int)h->ev.size() < 2 * pairs) {
                    hipEvent_t e;
                    HIPCHECK(hipEventCreate(&e));
                    h->ev.push_back(e);
                }
            }
            h->nrec = 0;
            h->tim_total_ms = 0.0;
            h->tim_last = 0;
            h->timing = true;
            return;
        }
        h->timing = false;
        if (launches) *launches = h->nrec;
        if (avg_ms) *avg_ms = h->nrec ? h->tim_total_ms / h->nrec : 0.0;
    });
}

mg_status mg_set_eager(mg_handle h, int eager) {
    if (!h) return MG_ERR_INVALID_ARG;
    h->eager = eager != 0;
    return MG_OK;
}

mg_status mg_destroy(mg_handle h) {
    if (!h) return MG_OK;
    std::lock_guard<std::mutex> lk(g_capture_mu);
    for (auto &e : h->ev) (void)hipEventDestroy(e);
    for (int p = 0; p < 3; ++p)
        for (int c = 0; c < 4; ++c) {
            if (h->iter_exec[p][c]) (void)hipGraphExecDestroy(h->iter_exec[p][c]);
            if (h->iter_graph[p][c]) (void)hipGraphDestroy(h->iter_graph[p][c]);
        }
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    for (void *p : h->allocs) (void)hipFree(p);
    if (h->host_scalar) (void)hipHostFree(h->host_scalar);
    delete h;
    return MG_OK;
}

const char *mg_last_error(void) { return g_last_error.c_str(); }

const char *mg_error_string(mg_status s) {
    switch (s) {
        case MG_OK: return "ok";
        case MG_ERR_INVALID_ARG: return "invalid argument";
        case MG_ERR_GEOMETRY: return "the grid does not resolve the geometry";
        case MG_ERR_SINGULAR: return "singular matrix";
        case MG_ERR_NO_CONVERGENCE: return "no convergence within max_iters";
        case MG_ERR_DIVERGED: return "the iteration diverged";
        case MG_ERR_OOM: return "out of device memory";
        case MG_ERR_HIP: return "HIP runtime error";
        case MG_ERR_UNSUPPORTED: return "unsupported configuration";
    }
    return "unknown status";
}

}  // extern "C"
