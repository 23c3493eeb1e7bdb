// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/svr.h"

namespace svr {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const char *fmt, ...);
void clear_error();

#define SVR_HIP(call)                                                             \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            ::svr::set_error("%s:%d %s: %s", __FILE__, __LINE__, #call,          \
                             hipGetErrorString(e_));                             \
            return e_ == hipErrorOutOfMemory ? SVR_ENOMEM : SVR_EDEVICE;          \
        }                                                                         \
    } while (0)

#define SVR_REQUIRE(cond, ...)                                                    \
    do {                                                                          \
        if (!(cond)) {                                                            \
            ::svr::set_error(__VA_ARGS__);                                        \
            return SVR_EINVAL;                                                    \
        }                                                                         \
    } while (0)

// Device allocations are stream-ordered (hipMallocAsync / hipFreeAsync) on the
// stream set by the innermost AllocStream of the calling thread, so creating
// or destroying an object never waits for work on other streams.  dmalloc
// honours an optional fault-injection budget (environment
// SVR_FAULT_ALLOC_AFTER=n makes the (n+1)-th allocation fail).
struct AllocStream {
    hipStream_t prev;
    explicit AllocStream(hipStream_t s);
    ~AllocStream();
};
hipError_t dmalloc(void **p, size_t bytes);
void dfree(void *p);

// Device blocks that a long-lived owner keeps for reuse instead of freeing them.  While a
// BlockCacheScope is active on the calling thread, dmalloc first takes an idle block of at least
// the size asked for and at most 5/4 of it, and records what it allocates; dfree of a recorded
// block keeps it idle when the scope was opened with keep = true (for objects whose work has
// completed on every stream), else frees it as usual.  Once more of the runtime's stream-ordered
// pool is free than in use, the runtime hands large blocks back to the driver as they are freed,
// at several ms a block with every host thread's calls held up; blocks kept here stay in use as
// far as the pool is concerned.
struct BlockCache {
    std::mutex mu;                           // scopes on several threads may share a cache
    std::unordered_map<void *, size_t> out;  // blocks handed out while a scope was active
    std::multimap<size_t, void *> idle;      // blocks kept, by size
    int64_t idle_bytes = 0;
    int64_t reuses = 0;
};
struct BlockCacheScope {
    BlockCache *prev_cache;
    bool prev_keep;
    BlockCacheScope(BlockCache *c, bool keep);
    ~BlockCacheScope();
};
// frees idle blocks, largest first, until at most max_idle bytes stay idle
void block_cache_trim(BlockCache &c, int64_t max_idle);
template <typename T>
inline hipError_t dalloc(T **p, size_t count) {
    return dmalloc(reinterpret_cast<void **>(p), count * sizeof(T));
}

// ---------------------------------------------------------------------------
// weights
// ---------------------------------------------------------------------------
// bf16 is stored as raw uint16_t; fp16 as _Float16.
struct bf16_t { uint16_t bits; };

__host__ __device__ inline float load_w(float v) { return v; }
__host__ __device__ inline float load_w(_Float16 v) { return static_cast<float>(v); }
__host__ __device__ inline float load_w(bf16_t v) {
    return __uint_as_float(static_cast<uint32_t>(v.bits) << 16);
}

// ---------------------------------------------------------------------------
// matrix object
// ---------------------------------------------------------------------------

// Zero entries after the last non-zero of every index and weight array, so
// that a batch of loads may run past the end of the last row: the kernels
// load unconditionally (a load behind a per-lane branch costs a wait for it
// before the branches join) and select valid entries afterwards.
constexpr int64_t NNZ_PAD = 1024;

// Tiled pixel order of the image the single-slice forward projection
// gathers from: 4 x 8-pixel tiles (one 128-byte cache line of FP32 values
// each), tiles row-major, pixels row-major within a tile.  A ray crosses a
// tile in several consecutive entries, so a wavefront's gathers touch far
// fewer cache lines than in row-major order (about 2.6x fewer at 256^2).
constexpr int TILE_W = 4, TILE_H = 8;
// XCDs of the device: workgroups are dispatched to them round-robin by index
constexpr int XCDS = 8;
__host__ __device__ inline int tiles_x(int nx) { return (nx + TILE_W - 1) / TILE_W; }
__host__ __device__ inline int tiled_count(int nx, int ny) {
    return tiles_x(nx) * TILE_W * ((ny + TILE_H - 1) / TILE_H) * TILE_H;
}
__host__ __device__ inline int tiled_index_xy(int ix, int iy, int tx) {
    return ((iy / TILE_H) * tx + ix / TILE_W) * (TILE_W * TILE_H) + (iy % TILE_H) * TILE_W + (ix % TILE_W);
}
// Whether a forward pass over `rows` rows runs a pair of rows per wavefront
// (32 lanes each) instead of one: when it has more rows than `pair_rows`
// (Matrix::pair_rows_eff: by default twice the wavefronts the device holds
// at once, 8 per SIMD).
__host__ __device__ inline bool forward_pairs_for(int64_t rows, int64_t pair_rows) { return rows > pair_rows; }
__host__ __device__ inline int tiled_index(int n, int nx, int tx) {
    const int iy = n / nx, ix = n - iy * nx;
    return tiled_index_xy(ix, iy, tx);
}
struct Matrix {
    svr_geometry geom;
    int Ns = 0, wtype = 0;
    int M = 0, N = 0;
    int64_t nnz = 0;
    int max_row_nnz = 0, max_col_nnz = 0;
    int device = 0;
    hipStream_t owner = nullptr;    // stream its memory was allocated on (freed there)
    std::vector<int> row_start;     // host, Ns+1: first subset-ordered row of each subset
    std::vector<int64_t> nnz_sub;   // host, Ns
    int *d_row_start = nullptr;     // device copy of row_start
    int *d_row_sino = nullptr;      // M: natural sinogram index of each subset-ordered row
    int *d_row_ptr = nullptr;       // M+1
    void *d_col = nullptr;          // nnz pixel indices (int32, or uint16 when idx16)
    void *d_colt = nullptr;         // the same in tiled pixel order (single-slice forward passes)
    int Nt = 0, tx = 0;             // tiled image size (>= N) and tiles per image row
    void *d_val = nullptr;          // nnz (float / _Float16 / bf16_t)
    int *d_ptrT = nullptr;          // Ns*N+1
    void *d_rowT = nullptr;         // nnz subset-local rows (int32, or uint16 when idx16)
    void *d_valT = nullptr;         // nnz
    int idx16 = 0;                  // indices stored as uint16 (N and every subset's rows <= 65536)
    float *d_sens_t = nullptr;      // Ns*N
    double *d_sens = nullptr;       // N
    int64_t bytes = 0;
    int cus = 0;                    // compute units of the device (sizes the whole-matrix runs)
    int pair_rows = 0;              // forward passes over more rows run in row pairs (0: 2 * 32 * cus)
    int pair_rows_eff() const { return pair_rows > 0 ? pair_rows : 2 * 32 * (cus > 1 ? cus : 1); }
    int run_fwd = 0;                // row pairs per wavefront in whole-matrix forward passes (0: by size)
    int run_bp = 0;                 // transposed rows per lane group in whole-matrix back-projections (0: by size)
    int xcd_bands = 1;              // one-row-per-wavefront forward passes: each XCD a band of bins (band_row)
    int sub_fwd_u = 0;              // one-row-per-wavefront forward passes: index/weight loads per lane and batch
                                    // (0: FWD_U; tuned among 4, 6, 8)
    int sub_bp_u = 0;               // per-subset update: loads per lane and batch (0: BP_U; tuned among 3, 4, 5, 6, 8)
    // scratch of the projector calls (svr_project / svr_backproject), max(Nt, M) floats kept
    // between calls: a call takes it when it is idle and its last use was on the call's stream
    // or has completed (proj_done), else allocates its own
    mutable float *proj_scratch = nullptr;
    mutable hipStream_t proj_stream = nullptr;
    mutable hipEvent_t proj_done = nullptr;
    mutable bool proj_busy = false;
    std::mutex *proj_mu = nullptr;  // created with the matrix
    int wbytes() const { return wtype == SVR_W_F32 ? 4 : 2; }
    int ibytes() const { return idx16 ? 2 : 4; }
    int rows_of(int t) const { return row_start[t + 1] - row_start[t]; }
};

// Calls f(WT{}, IT{}) with the matrix's weight and index storage types.
template <class F>
inline int with_types(const Matrix &A, F &&f) {
    if (A.idx16) {
        if (A.wtype == SVR_W_F32) return f(float{}, uint16_t{});
        if (A.wtype == SVR_W_F16) return f(_Float16{}, uint16_t{});
        return f(bf16_t{}, uint16_t{});
    }
    if (A.wtype == SVR_W_F32) return f(float{}, int{});
    if (A.wtype == SVR_W_F16) return f(_Float16{}, int{});
    return f(bf16_t{}, int{});
}

// ---------------------------------------------------------------------------
// kernel launchers (defined next to their kernels)
// ---------------------------------------------------------------------------

// geometry / build
int build_matrix(Matrix &A, const float *mu_dev, hipStream_t s);

// forward projection of rows [r0, r1) of the subset-ordered matrix.
//  mode 0: y[row_sino[r]] = (A f)_r                           (plain projection)
//  mode 1: ratio[r] = g[r] / ((A f)_r + w[r])   (0 if g == 0 or ybar <= 0)
//  mode 2: log-likelihood term of row r into part[r - r0], ratio not written
//          (*n_blocks_out receives the number of terms, r1 - r0)
struct FwdArgs {
    const float *f;       // image in tiled order (Nt floats; slice stacks: [N][S] natural)
    const float *g, *w;   // subset-ordered data (modes 1, 2)
    float *out;           // mode 0: natural-order sinogram; mode 1: ratio (subset order)
    double *part;         // mode 2: one term per row
    int *bad;             // mode 2: set when g > 0 and ybar <= 0
    double eps = 0.0;     // > 0: modified likelihood for rows with w = 0 and ybar <= eps
};
int launch_forward(const Matrix &A, int r0, int r1, int mode, const FwdArgs &a, hipStream_t s,
                   int *n_blocks_out = nullptr);

// back-projection of subset t (or all subsets with t = -1) of a ratio/data
// vector in subset-ordered rows: x[n] = sum over the transposed row.
int launch_backproject(const Matrix &A, int t, const float *y_sub, float *x, hipStream_t s);

// ft[tiled(n)] = f[n] (the pad entries of ft are left as they are)
int launch_tile_image(const Matrix &A, const float *f, float *ft, hipStream_t s);

// deterministic FP64 reduction of n partials into out[0]
int launch_reduce_sum(const double *part, int n, double *out, hipStream_t s);

// penalty value partials (FP64): R(f) for one slice image
int launch_penalty_value(const Matrix &A, const float *f, int potential, double delta,
                         double *part, int *n_blocks_out, hipStream_t s);

// permute natural-order sinogram into subset order (and back)
int launch_gather_rows(const Matrix &A, const float *src_nat, float *dst_sub, hipStream_t s);

// validation counters: counts entries that are negative / non-finite / non-positive
int launch_count_bad(const float *x, int64_t n, int require_positive, int *counter, hipStream_t s);

// ---------------------------------------------------------------------------
// per-pixel fused updates (update.hip)
// ---------------------------------------------------------------------------
struct PenaltyArgs {
    int potential;
    double delta;
    double beta;
    int nx, ny;
};

struct UpdateArgs {
    int t;                   // subset
    int Ns;
    const float *ratio;      // ratio of subset t (subset-local rows)
    const float *f;          // current image f^k
    float *f_out;            // f^{k+1}
    double alpha;
    // algorithm state
    double *s_hat;           // SVREM/SEM running statistic (N)
    const double *s_anc;     // SVREM anchor statistic (N)
    float *table;            // Ns*N table (SVREM tau_anc, SVRG q_anc, SAGA q)
    double *Q;               // SAGA running table sum (N)
    const double *g_tilde;   // SVRG anchor full gradient / Ns (N)
    const float *dpre;       // frozen preconditioner (N or Ns*N), null for iterate mode
    int dpre_per_subset;     // 1 if dpre is Ns*N
    int shat_zero;           // SEM first step: the previous s_hat is taken as 0
    PenaltyArgs pen;
    int t2;                  // SAGA-EM: refreshed subset (t2 == t: the same back-projection)
    const float *ratio2;     // SAGA-EM: ratio of subset t2 (subset-local rows)
    float *ft_out;           // f^{k+1} also in tiled order for the next forward pass (nullable)
    int tx;                  // tiles per image row
};

enum UpdateKind { UPD_OSEM = 0, UPD_SVREM = 1, UPD_SVRG = 2, UPD_SAGA = 3, UPD_SGA = 4, UPD_SEM = 5,
                  UPD_SAGAEM = 6 };
int launch_update(const Matrix &A, int kind, const UpdateArgs &u, hipStream_t s);

// anchor (snapshot) pass at the current image, with the ratio of every row
// (subset-ordered) already computed.
//  table kernel: one entry per (subset t, pixel n):
//    SVREM, SAGA-EM: tau_t[n] = Ns f_n b_t[n];  SVRG/SAGA: q_t[n] = b_t[n] - beta/Ns grad R(f)_n
//  sum kernel (fixed t order, FP64):
//    SVREM: s_anc = mean_t tau_t (and s_hat = s_anc if init_shat)
//    SAGA-EM: Q = sum_t tau_t, s_hat = Q / Ns
//    SVRG : g_tilde = (sum_t q_t - A^T 1) / Ns
//    SAGA : Q = sum_t q_t
struct SnapArgs {
    const float *ratio_all;
    const float *f;
    float *table;
    double *s_anc;
    double *s_hat;
    int init_shat;
    double *g_tilde;
    double *Q;
    PenaltyArgs pen;
    // SVRG / SAGA: grad R(f)_n per pixel, computed once for the table (every
    // subset's entry of pixel n carries the same term); nullptr: each entry
    // computes it from f itself (the same function on the same values)
    const double *grad;
};
// grad R(f)_n of every pixel (the penalty of `p`) into out[N]
int launch_penalty_grad(const Matrix &A, const float *f, const PenaltyArgs &p, double *out, hipStream_t s);
int launch_anchor_table(const Matrix &A, int kind, const SnapArgs &a, hipStream_t s);
int launch_anchor_sum(const Matrix &A, int kind, const SnapArgs &a, hipStream_t s);
// anchor sums fused with the update of the iteration that takes the anchor
int launch_anchor_sum_update(const Matrix &A, int kind, const SnapArgs &a, const UpdateArgs &u, hipStream_t s);

// persistent epoch kernel (persist.hip): a whole epoch call in one
// cooperative launch
struct EpochArgs {
    const int *row_ptr;
    const void *col;
    const void *val;
    const int *ptrT;
    const void *rowT;
    const void *valT;
    const int *row_start;
    const float *sens_t;
    const double *sens;
    int M, N, Ns;
    int pair_rows;  // forward phases over more rows run in pairs (forward_pairs_for)
    const float *g, *w;
    float *ratio;
    float *f0, *f1;
    int cur0;
    float *ft;   // the iterate in tiled order: read by the forward phases, written by the updates
    int tx;
    double eps;  // modified likelihood (0: off)
    double *s_hat, *s_anc, *Q, *g_tilde;
    float *table;
    float *dpre;
    int dpre_per_subset;
    PenaltyArgs pen;
    double alpha, decay;
    int decaying, eta, flags;
    const int *order;
    int n;
    long long k0;
    unsigned *sync;
    int *status;
};
int launch_epoch(const Matrix &A, int kind, const EpochArgs &e, hipStream_t s, int *grid_cache);
int persistent_sync_words();

// slice stacks (slices.hip): images [N][S], data and ratios [row][S]
//
// The image is cut into a grid of rectangular regions (ry x rx, each ly x lx
// pixels, the last ones smaller) small enough that one region of the stack,
// ly * lx * S floats, fits in an XCD's L2 with room to spare.  Region q belongs
// to XCD q mod XCDS (workgroups are dispatched to the XCDs round-robin by
// index).  A ray crosses a convex region in one run of consecutive entries of
// its row, so each row splits into segments, one per region it crosses, in ray
// order.
struct Regions {
    int ry = 1, rx = 1, ly = 1, lx = 1;
};
struct XcdSched {  // per XCD: first entry in a schedule and number of entries
    int off[XCDS];
    int cnt[XCDS];
};
struct StackPlan {
    Regions reg;
    int S = 0, nch = 0;
    int64_t nseg = 0;
    int *seg_ptr = nullptr;      // M+1: segments of subset-ordered row r are [seg_ptr[r], seg_ptr[r+1])
    int *seg_beg = nullptr;      // nseg+1: first entry of each segment (seg_beg[nseg] = nnz)
    int *sched_sub = nullptr;    // nseg: each subset's segments grouped by XCD, region-major
    int *sched_all = nullptr;    // nseg: every segment grouped by XCD, region-major
    std::vector<XcdSched> sub;   // per subset, offsets into sched_sub
    XcdSched all{};              // offsets into sched_all
    int area[XCDS] = {};         // pixels of each XCD's regions
    double *P = nullptr;         // nseg x (64 nch) FP64 segment sums
};
Regions choose_regions(int nx, int ny, int S);
int ms_plan_build(const Matrix &A, int S, StackPlan &plan, hipStream_t s);
void ms_plan_free(StackPlan &plan);
// mode 1: ratio of every row of subset t (t = -1: all rows); mode 2: the
// log-likelihood partials of all rows (t = -1), *nb_out of them in part
int ms_forward(const Matrix &A, const StackPlan &plan, int t, int mode, int S, const float *X, const float *g,
               const float *w, float *ratio, double *part, int *bad, hipStream_t s, int *nb_out);
int ms_update(const Matrix &A, const StackPlan &plan, int kind, int S, int axial, const UpdateArgs &u, hipStream_t s);
int ms_anchor_table(const Matrix &A, const StackPlan &plan, int S, const float *ratio_all, const float *X,
                    float *table, hipStream_t s);
int ms_anchor_sum(const Matrix &A, int S, const float *table, double *s_anc, double *s_hat, int init_shat,
                  hipStream_t s);
int ms_penalty_value(const Matrix &A, int S, const float *X, int potential, double delta, int axial, double *part,
                     int *nb_out, hipStream_t s);
int ms_pack_sino(const Matrix &A, int S, const float *src, float *dst, hipStream_t s);
int ms_pack_img(int N, int S, const float *src, float *dst, hipStream_t s);
int ms_unpack_img(int N, int S, const float *src, float *dst, hipStream_t s);

// frozen preconditioner d = f0 / sens_t (per subset) or f0 / sens
int launch_precond(const Matrix &A, const float *f0, int per_subset, float *d, hipStream_t s);

}  // namespace svr

struct svr_matrix : public svr::Matrix {};
