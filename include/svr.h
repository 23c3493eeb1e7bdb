/*
 * svr.h -- C ABI of the MI355X variance-reduced stochastic EM library.
 *
 * The library reconstructs images from Poisson emission data with the model
 * of Kereta, Twyman, Arridge, Thielemans and Jin, "Stochastic EM methods with
 * variance reduction for penalised PET reconstructions" (arXiv:2106.03172):
 *
 *   E[g] = A f + w                      (Sec. 2.1, eq. voxel_td)
 *   Phi(f) = L(f) - beta R(f), f >= 0   (Sec. 3, eq. PET-MAP)
 *
 * with an ordered-subset partition of the data (Sec. 2.1), the OSEM update
 * (Sec. 2.2), SVREM (Sec. 2.3, eq. tempsvrem, with the penalised M-step of
 * Sec. 3), the preconditioned SAGA and SVRG updates (Sec. 4, eq. saga_update
 * and svrg_update) and the SGA, BSREM and SEM baselines (Sec. 4, Sec. 5.1).
 *
 * Conventions shared by every call:
 *  - Every call returns an int status (SVR_OK = 0, negative on error); no
 *    C++ exception crosses the ABI.  svr_last_error() returns a thread-local
 *    message describing the last non-OK status of the calling thread.
 *  - "_dev" pointers are device memory on the current HIP device, borrowed
 *    from the caller: they must stay valid until the work enqueued on the
 *    given stream has completed.  Host arrays are copied before return.
 *  - "stream" is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls that only enqueue work return before it completes; calls
 *    documented as "synchronises" wait for the stream.
 *  - Opaque handles are owned by the library and released with *_destroy
 *    (NULL-safe).  A handle must not be used from two threads at once.
 *  - Sinograms are float32 in natural order [slice][view][bin]
 *    (m = v*B + b); images are float32 [slice][iy][ix] (n = iy*nx + ix).
 *  - Invalid arguments return SVR_EINVAL before anything is enqueued.
 */
#ifndef SVR_H
#define SVR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define SVR_OK          0
#define SVR_PENDING     1   /* serving: request not finished yet */
#define SVR_EINVAL     -1   /* invalid argument or state */
#define SVR_ENOMEM     -2   /* device or host allocation failed */
#define SVR_EDEVICE    -3   /* HIP runtime error */
#define SVR_ENOTFOUND  -4   /* unknown ticket */
#define SVR_ENUMERIC   -5   /* non-finite objective or data */
#define SVR_ECANCELLED -6   /* request cancelled */

/* Message for the last non-OK status returned on this thread ("" if none). */
const char *svr_last_error(void);
/* Library ABI version (major*10000 + minor*100 + patch). */
int svr_version(void);

/* ---- geometry and system matrix ----------------------------------------- */

/* 2D parallel-beam scanner.  View v has angle v*arc_rad/n_views; bin b sits
 * at radial offset (b - (n_bins-1)/2)*bin_mm; the image grid has nx*ny square
 * pixels of pixel_mm centred on the rotation axis.  The paper leaves the
 * projector open (Sec. 2.1 only asks for a non-negative A); this library uses
 * exact ray/pixel intersection lengths in mm (Siddon's method), computed in
 * FP64 with half-open pixels, axis-snapped views (|cos|,|sin| < 1e-12 -> 0)
 * and pieces shorter than 1e-9 pixel dropped. */
typedef struct {
    int32_t nx, ny;
    double  pixel_mm;
    int32_t n_views, n_bins;
    double  bin_mm;
    double  arc_rad;     /* angular range, normally pi */
} svr_geometry;

/* Storage type of the matrix weights.  Products are accumulated in FP64
 * whatever the storage type.  Index arrays are uint16 when every pixel index
 * and every subset-local row index fits (N <= 65536 and at most 65536 rows per
 * subset), else int32; OR-ing SVR_W_INDEX32 into wtype forces int32. */
enum { SVR_W_F32 = 0, SVR_W_F16 = 1, SVR_W_BF16 = 2 };
#define SVR_W_INDEX32 0x100

typedef struct svr_matrix svr_matrix;
typedef struct svr_recon  svr_recon;
typedef struct svr_server svr_server;

/* Builds A on the device (Sec. 2.1, eq. voxel_td) together with its ordered
 * subsets (Sec. 2.1): subset t holds the views v = t (mod n_subsets), and its
 * rows are stored view-major, bin-minor.  Two layouts are kept: the rows of A
 * in subset order (forward projection) and, per subset, the transposed rows
 * (one per pixel, entries by ascending view and bin) for a gather-only
 * back-projection.  Also computes the sensitivities A_t^T 1 and A^T 1.
 *   geom        : scanner; nx, ny, n_views, n_bins >= 1, sizes > 0
 *   n_subsets   : 1 <= n_subsets <= n_views, n_subsets * nx * ny < 2^31
 *   wtype       : SVR_W_F32 / SVR_W_F16 / SVR_W_BF16 (round to nearest even)
 *   mu_dev      : optional attenuation map (nx*ny floats, 1/mm, >= 0) or NULL;
 *                 every weight of ray m is multiplied by exp(-sum_n a_mn mu_n)
 *   stream      : work is enqueued there; the call synchronises before return
 *   out         : receives the new handle (release with svr_matrix_destroy)
 * Errors: SVR_EINVAL (bad sizes, nnz beyond int32), SVR_ENOMEM, SVR_EDEVICE. */
int svr_build_system_matrix(const svr_geometry *geom, int32_t n_subsets, int32_t wtype,
                            const float *mu_dev, void *stream, svr_matrix **out);

typedef struct {
    int64_t nnz;           /* non-zeros of A */
    int64_t bytes;         /* device bytes held by the matrix object */
    int32_t n_subsets;
    int32_t n_rows;        /* M = n_views * n_bins */
    int32_t n_pixels;      /* N = nx * ny */
    int32_t max_row_nnz;   /* longest row of A */
    int32_t max_col_nnz;   /* longest transposed row of any subset */
    int32_t wtype;         /* SVR_W_F32 / F16 / BF16 */
    int32_t index_bytes;   /* 2 (uint16) or 4 (int32) */
} svr_matrix_info_t;

/* Sizes of a built matrix; nnz_per_subset (nullable) receives n_subsets
 * counts.  Synchronous, host-only. */
int svr_matrix_info(const svr_matrix *A, svr_matrix_info_t *info, int64_t *nnz_per_subset);

/* Copies one layout of A to host buffers, for inspection and tests.
 *   which = 0: rows of A in natural sinogram order (row m = v*B + b):
 *              ptr[M+1], idx[nnz] = pixel, val[nnz] as float
 *   which = 1: transposed rows, subset-major: ptr[Ns*N+1], row (t*N + n)
 *              lists idx = subset-local row (view-major, bin-minor), val
 * Any of ptr/idx/val may be NULL to skip it.  Synchronises. */
int svr_matrix_export(const svr_matrix *A, int32_t which, int32_t *ptr, int32_t *idx, float *val);

/* Sensitivity A_t^T 1 (subset >= 0, stored FP32 from an FP64 sum) or A^T 1
 * (subset = -1, FP64) into out_dev (N doubles). */
int svr_sensitivity(const svr_matrix *A, int32_t subset, double *out_dev, void *stream);

void svr_matrix_destroy(svr_matrix *A);

/* Run lengths of the passes over the whole matrix (the anchor pass of
 * eq. tempsvrem / eq. svrg_update / eq. saga_update, the objective, and the
 * projectors over all subsets).  A forward wavefront sums a pair of
 * consecutive rows (32 lanes each); one that owns a run of pairs keeps the
 * next pair's loads in flight while it sums the current one; the run length
 * never changes a row's arithmetic, so every result is bitwise the same under
 * any tuning.  0 means "chosen from the sizes and the device's compute units".
 * A forward pass over no more row pairs than the device holds wavefronts at
 * once (the per-subset passes at the usual sizes) always runs one pair per
 * wavefront. */
typedef struct {
    int32_t fwd_pairs_per_wave;  /* pairs of rows of A per wavefront, 0..31 */
    int32_t bp_rows_per_group;   /* (subset, pixel) transposed rows per lane group, 0..1024 */
    int32_t fwd_pair_rows;       /* forward passes over more rows than this run a pair of rows per
                                    wavefront, others one row (0: twice the wavefronts the device
                                    holds at once, 2 * 32 * compute units); >= 0 */
    double  fwd_us, bp_us;       /* svr_matrix_tune: measured duration of the chosen runs */
    int32_t fwd_natural_order;   /* forward passes with one row per wavefront (the per-subset passes):
                                    0 (default) gives each of the device's 8 XCDs a band of bins of every
                                    view, so its L2 holds the part of the image those rays cross; 1 takes
                                    the rows in order.  Results are bitwise the same either way. */
    int32_t subset_fwd_batch;    /* per-subset forward passes with one row per wavefront: index/weight
                                    loads per lane issued together, 4, 6 or 8 (0: 8) */
    int32_t subset_bp_batch;     /* per-subset update: loads per lane of each pixel's 4-lane group issued
                                    together, 3, 4, 5, 6 or 8 (0: 5).  Neither width changes the entries
                                    a lane adds or their order, so results are bitwise the same. */
} svr_tuning_t;

/* Run lengths and batch widths in use (0 resolved to the size-based or
 * default choice); fwd_us and bp_us are 0.  Host-only. */
int svr_matrix_get_tuning(const svr_matrix *A, svr_tuning_t *t);

/* Sets the run lengths (0 = size-based) and batch widths (0 = default).
 * Errors: SVR_EINVAL out of range.
 * Not to be called while work that uses A is being enqueued from another
 * thread. */
int svr_matrix_set_tuning(svr_matrix *A, const svr_tuning_t *t);

/* Autotuner: times the candidate run lengths of the whole-matrix forward
 * pass and of the anchor table on A itself, the two kernels alternating as in
 * an anchor pass (HIP events on `stream`, median of 9 pairs, synthetic
 * operands), then the batch widths of the per-subset forward and SVREM update
 * passes, timed together over all subsets as an epoch runs them (median of 9;
 * the default widths are kept unless a pair is at least 2% faster), keeps the
 * fastest in A and reports them in out (nullable).
 * Allocates about 4(2M + N + Ns*N) bytes for the duration of the call and
 * synchronises.  With the environment variable SVR_TUNE_CACHE naming a file,
 * a matrix whose geometry, subsets, weight and index types and device (name,
 * compute units) are recorded there takes the recorded choices without
 * timing (out reports the recorded durations); otherwise the result is
 * appended to the file (one text line per tuning; unreadable lines are
 * ignored, an unwritable file only costs the next call its timing).
 * Errors: SVR_ENOMEM, SVR_EDEVICE (A unchanged). */
int svr_matrix_tune(svr_matrix *A, void *stream, svr_tuning_t *out);

/* ---- projectors ---------------------------------------------------------- */

/* Forward projection y = A_t x (subset t; subset = -1: all of A).  Only the
 * bins of subset t are written; others are left untouched.
 *   x_dev : [n_slices][N] floats;  y_dev : [n_slices][M] floats (natural order) */
int svr_project(const svr_matrix *A, int32_t subset, const float *x_dev, int32_t n_slices,
                float *y_dev, void *stream);

/* Back-projection x = A_t^T y over the bins of subset t (subset = -1: A^T y).
 * x_dev is overwritten.  Gather-only and deterministic (fixed summation order). */
int svr_backproject(const svr_matrix *A, int32_t subset, const float *y_dev, int32_t n_slices,
                    float *x_dev, void *stream);

/* Forward projection exactly as svr_project (same kernels, bitwise the same
 * result), for callers that cannot allocate device memory: code under HIP
 * graph capture, serving loops and harnesses that forbid hipMalloc.  The call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine): the
 * tiled copy of each slice goes to a scratch array of
 * SVR_NOALLOC_SCRATCH_FLOATS floats (4 MiB) that the library keeps in device
 * memory on every device it runs on until the process ends.  The tiled image,
 * ceil(nx/4)*4 * ceil(ny/8)*8 floats, must fit (up to 1024 x 1024).
 * Every call on one device shares that array: calls that overlap on one GPU
 * (two streams, or two host threads) race on it and must be serialised by the
 * caller.  Nothing in the array needs to start at zero (each call writes every
 * slot it reads).
 * Errors: SVR_EINVAL (NULL, subset out of range, n_slices < 1, tiled image
 * beyond the scratch), SVR_EDEVICE. */
#define SVR_NOALLOC_SCRATCH_FLOATS (1 << 20)
int svr_project_noalloc(const svr_matrix *A, int32_t subset, const float *x_dev, int32_t n_slices,
                        float *y_dev, void *stream);

/* ---- reconstruction ------------------------------------------------------ */

enum { SVR_ALGO_OSEM = 0, SVR_ALGO_SVREM = 1, SVR_ALGO_SVRG = 2, SVR_ALGO_SAGA = 3,
       SVR_ALGO_SGA = 4, SVR_ALGO_BSREM = 5, SVR_ALGO_SEM = 6, SVR_ALGO_SAGAEM = 7 };
/* Potentials of Table 1 (Sec. 3). */
enum { SVR_PEN_QUADRATIC = 0, SVR_PEN_HUBER = 1, SVR_PEN_LOGCOSH = 2, SVR_PEN_HYPERBOLA = 3 };
/* Preconditioner of SVRG and SAGA (Sec. 4, eq. preconditioners).  The
 * experiments of Sec. 5 freeze it at the first iteration, d = d(f0); Theorem 1
 * and Appendix B take one vector for every subset, f0 / A^T 1, which is the
 * default (0).  The subset-indexed frozen form is about Ns times larger, so it
 * needs a step about Ns times smaller than the paper's alpha = 2. */
enum { SVR_PRECOND_FULL_FROZEN   = 0,  /* d   = f0 / A^T 1   (default) */
       SVR_PRECOND_SUBSET_FROZEN = 1,  /* d_t = f0 / A_t^T 1 */
       SVR_PRECOND_ITERATE       = 2 };/* d_t = f^k / A_t^T 1 */
#define SVR_FLAG_RESET_SHAT_AT_ANCHOR 1 /* SVREM: s_hat = s_anc at every anchor */
#define SVR_FLAG_AXIAL_PENALTY        2 /* slices: add the 2 axial neighbours */
#define SVR_FLAG_PERSISTENT_EPOCH     4 /* run each epoch call as one persistent cooperative
                                           kernel with grid barriers instead of one kernel
                                           per phase (bitwise the same results) */
#define SVR_FLAG_MODIFIED_LL          8 /* SVRG, SAGA, SGA, BSREM: the modified likelihood of
                                           Sec. 2.3 (eq. modified_LL) -- rows with w = 0 and
                                           ybar <= ll_eps use the second-order expansion of
                                           g log ybar - ybar about ll_eps, in the gradient
                                           and in svr_objective */

typedef struct {
    int32_t algo;      /* SVR_ALGO_*: which state the recon keeps */
    double  alpha;     /* step size (> 0); BSREM/SEM: a_0 of a_k = alpha/(decay*k+1) */
    int32_t eta;       /* SVREM/SVRG anchor period in epochs (>= 1) */
    double  beta;      /* penalty strength (>= 0) */
    int32_t penalty;   /* SVR_PEN_* */
    double  delta;     /* potential parameter (> 0 for Huber/log cosh/hyperbola) */
    int32_t precond;   /* SVR_PRECOND_* (SVRG, SAGA) */
    int32_t flags;     /* SVR_FLAG_* */
    double  decay;     /* BSREM/SEM step decay (0.001 in the paper) */
    double  ll_eps;    /* eps of SVR_FLAG_MODIFIED_LL (> 0 when the flag is set) */
} svr_params;

/* Creates a reconstruction of n_slices images that share A (the slices are
 * coupled only by the optional axial penalty).  g, w and f0 are copied.
 * With n_slices > 1 the data are processed as one sparse-times-dense product
 * per subset (slices as columns) and the recon runs OSEM and SVREM epochs
 * (other algos are rejected with SVR_EINVAL).  SVR_FLAG_MODIFIED_LL needs a
 * gradient algo (SVRG, SAGA, SGA, BSREM) and a finite ll_eps > 0; the
 * persistent flag is not available with SAGAEM.  A stack's image and
 * sinogram blocks (n_slices x N and n_slices x M floats) must each stay below
 * 2^31 bytes (SVR_EINVAL otherwise).
 *   g_dev  : [S][M] counts (finite, >= 0);  w_dev: [S][M] background (finite, >= 0)
 *   f0_dev : [S][N] starting image (finite, > 0)
 * The matrix must outlive the recon.  Synchronises (validates the data). */
int svr_recon_create(svr_matrix *A, const float *g_dev, const float *w_dev, const float *f0_dev,
                     int32_t n_slices, const svr_params *params, void *stream, svr_recon **out);

/* Epochs.  Each runs n subset updates with the subsets order[0..n-1] (host
 * array, entries in [0, n_subsets); the paper draws them uniformly at random,
 * which is left to the caller so that runs are reproducible).  The iteration
 * counter k persists across calls.
 *  osem : f <- f * A_t^T(g_t/(A_t f + w_t)) / A_t^T 1 (Sec. 2.2, eq. Mstep).
 *         Usable with every algo as the initialiser; it resets the
 *         variance-reduction state (k = 0) of the recon.
 *  svrem: at k mod (eta*Ns) == 0 stores tau_t(f) for all t and their mean
 *         s_anc (FP64) (Sec. 2.3, eq. tempsvrem); s_hat <- (1-alpha) s_hat
 *         + alpha (tau_t(f) - tau_t(f_anc) + s_anc); f <- penalised M-step root
 *         (Sec. 3, eq. svrsurder).  s_hat starts at s(f^0).
 *  svrg : preconditioned proximal SVRG (Sec. 4, eq. svrg_update) with the
 *         anchor gradient table refreshed at k mod (eta*Ns) == 0.
 *  saga : preconditioned proximal SAGA (Sec. 4, eq. saga_update); the table
 *         is filled at f^0 at k = 0.
 *  sga, bsrem, sem: the non-variance-reduced baselines of Sec. 5.1.
 * The call must match params.algo (osem excepted).  Enqueues only.
 * Errors: SVR_EINVAL (NULL recon, order outside [0, n_subsets), wrong algo),
 * SVR_ENUMERIC after a non-finite objective. */
int svr_osem_epoch (svr_recon *R, const int32_t *order, int32_t n, void *stream);
int svr_svrem_epoch(svr_recon *R, const int32_t *order, int32_t n, void *stream);
int svr_svrg_epoch (svr_recon *R, const int32_t *order, int32_t n, void *stream);
int svr_saga_epoch (svr_recon *R, const int32_t *order, int32_t n, void *stream);
int svr_sga_epoch  (svr_recon *R, const int32_t *order, int32_t n, void *stream);
int svr_bsrem_epoch(svr_recon *R, const int32_t *order, int32_t n, void *stream);
int svr_sem_epoch  (svr_recon *R, const int32_t *order, int32_t n, void *stream);

/* SAGA-type online EM (Sec. 2.3, the remark after eq. tempsvrem): a table
 * S_t of subset statistics (FP32, filled with tau_t(f^0) for every t at k = 0,
 * with s_hat^0 = mean_t S_t) and its FP64 sum Q.  Iteration k on subset
 * t = order[i] with refreshed index t~ = refresh[i]:
 *   s_hat <- (1-alpha) s_hat + alpha (tau_t(f) - S_t + Q/Ns);
 *   S_t~ <- tau_t~(f), Q += tau_t~(f) - S_t~ (f the image before the update);
 *   f <- penalised M-step root (Sec. 3).
 * refresh (host array of n entries in [0, n_subsets)) may be NULL: t~ = t.
 * A t~ different from t costs a second subset projection.  Enqueues only;
 * errors as for the other epoch calls. */
int svr_sagaem_epoch(svr_recon *R, const int32_t *order, const int32_t *refresh, int32_t n, void *stream);

/* Phi(f) = sum_m g_m log(ybar_m) - ybar_m - beta R(f), ybar = A f + w, in FP64
 * over all slices (Sec. 3, eq. PET-MAP; 0 log 0 = 0; with SVR_FLAG_MODIFIED_LL
 * the modified terms of eq. modified_LL).  Synchronises.
 * Returns SVR_ENUMERIC (and marks the recon) if Phi is not finite. */
int svr_objective(svr_recon *R, double *phi_host, void *stream);

/* Copies the current image ([S][N] floats) to f_dev. */
int svr_get_image(const svr_recon *R, float *f_dev, void *stream);

typedef struct {
    int64_t k;                /* subset updates since the last reset */
    int64_t n_snapshots;      /* full passes taken (anchors, table fills) */
    int32_t n_subsets, n_slices, n_pixels, n_rows;
    int64_t state_bytes;      /* size of a svr_recon_get_state buffer */
} svr_recon_info_t;
int svr_recon_info(const svr_recon *R, svr_recon_info_t *info);

/* Checkpoint: serialises the whole algorithm state (iterate, running
 * statistics, anchors, tables, counters) to a host buffer.  get_state with
 * buf = NULL reports the size in *len.  A state restored with set_state
 * into a recon created with the same matrix, data and params continues
 * bitwise as the uninterrupted run.  Both synchronise. */
int svr_recon_get_state(const svr_recon *R, void *buf, size_t *len, void *stream);
int svr_recon_set_state(svr_recon *R, const void *buf, size_t len, void *stream);

void svr_recon_destroy(svr_recon *R);

/* Kernel timing (measurement aid).  While enabled, every kernel launch of the
 * epoch calls is bracketed by two HIP events recorded on the caller's stream;
 * svr_recon_kernel_times synchronises, reports per-kernel launch counts and
 * summed durations since the last report, and resets them.  Kinds:
 *   0 forward projection + EM ratio of one subset
 *   1 fused back-projection + update of one subset
 *   2 forward projection + EM ratio of all rows (anchor / table fill)
 *   3 anchor back-projection of every (subset, pixel) into the table
 *   4 anchor FP64 sums over the table (s_anc, g_tilde or Q)
 *   5 persistent epoch kernel (one per epoch call; kinds 0-4 then stay 0)
 * For kinds 0-4 the events are attached to the kernel dispatch itself, so
 * they time the kernel's execution as a profiler does; kind 5 is bracketed
 * by events recorded on the stream just before and after its launch. */
#define SVR_NUM_KERNEL_KINDS 6
typedef struct {
    int64_t launches[SVR_NUM_KERNEL_KINDS];
    double  total_ms[SVR_NUM_KERNEL_KINDS];
} svr_kernel_times_t;
int svr_recon_set_profiling(svr_recon *R, int32_t enable);
int svr_recon_kernel_times(svr_recon *R, svr_kernel_times_t *out);

/* ---- serving -------------------------------------------------------------- */

/* A continuous-batching server for independent SVREM reconstruction requests
 * of different sizes.  Requests are admitted while their device footprint
 * fits in the memory budget and a slot is free; every scheduler tick advances
 * each resident request by one epoch of subset updates.  With batch = 1 the
 * subset iterations of all resident requests with the same weight and index
 * types run as one forward and one update launch per iteration (work items
 * (request, row block) and (request, pixel block), up to 8 requests a launch;
 * the requests at an anchor as one whole forward, one table and one
 * anchor-sums + update launch); with batch = 0 each request's epoch is
 * enqueued on one of the streams so that requests overlap.  A request's
 * result does not depend on which other requests share the device, nor on
 * batch. */
typedef struct {
    int64_t mem_budget_bytes;  /* device bytes the server may hold (> 0) */
    int32_t max_slots;         /* max resident requests (>= 1) */
    int32_t n_streams;         /* device streams (>= 1): matrix builds, and per-request epochs when batch = 0 */
    int32_t batch;             /* 1: batched subset iterations (requests may not set
                                  SVR_FLAG_PERSISTENT_EPOCH); 0: one request's epoch per stream */
    int32_t share_matrices;    /* 1: requests with the same geometry, subset count and weight
                                  type use one matrix, built once and kept on the device after
                                  its last user finishes while the budget allows (a later
                                  request of that key skips the build); 0: each request builds
                                  its own */
} svr_serve_config;

typedef struct {
    svr_geometry geom;
    int32_t n_subsets;
    int32_t wtype;
    svr_params params;         /* algo must be SVR_ALGO_SVREM */
    int32_t epochs;            /* SVREM epochs after one OSEM initialisation epoch */
    uint64_t order_seed;       /* seeds the library's own subset sequence */
    const float *g_host;       /* [M] counts, copied at submit */
    const float *w_host;       /* [M] background, copied at submit */
    float f0_value;            /* constant starting image (> 0) */
} svr_serve_request;

typedef struct {
    float *f_host;             /* caller buffer of N floats, filled when done */
    double phi;                /* final objective */
    double queue_ms, run_ms;   /* time waiting for admission, time resident */
    int32_t status;            /* SVR_OK / SVR_ENUMERIC / SVR_ECANCELLED ... */
} svr_serve_result;

int  svr_serve_create(const svr_serve_config *cfg, svr_server **out);
/* Copies the request and queues it; rejects (SVR_EINVAL) a request that can
 * never fit the memory budget. */
int  svr_serve_submit(svr_server *S, const svr_serve_request *req, uint64_t *ticket);
/* Runs scheduler ticks for up to max_ticks (0 = until every admitted request
 * has finished) and admits queued requests as memory frees up. */
int  svr_serve_step(svr_server *S, int32_t max_ticks);
/* SVR_PENDING until the request is done; then fills *res (f_host, if not NULL,
 * must point to N floats: the final image, zeros for a request cancelled or
 * failed before it had one) and forgets the ticket. */
int  svr_serve_poll(svr_server *S, uint64_t ticket, svr_serve_result *res);
/* Host-only: writes up to cap tickets of finished requests whose results are
 * not yet polled (ascending ticket order) to tickets[] and their number to *n,
 * so that a caller polls only those.  Errors: SVR_EINVAL (NULL S or n, cap < 0,
 * NULL tickets with cap > 0). */
int  svr_serve_done(const svr_server *S, uint64_t *tickets, int32_t cap, int32_t *n);
int  svr_serve_cancel(svr_server *S, uint64_t ticket);
void svr_serve_destroy(svr_server *S);

/* Server state for monitoring (host-only, enqueues nothing): queue depth,
 * slots in use, device memory held, and running totals. */
typedef struct {
    int32_t queued;            /* submitted, waiting for admission */
    int32_t resident;          /* admitted and iterating (<= max_slots) */
    int32_t max_slots;
    int32_t done_unpolled;     /* finished (any status), result not yet polled */
    int64_t used_bytes;        /* device bytes held by resident requests: the recons' estimates
                                  and the matrices they use, each matrix once (its estimate until
                                  it is built, then its actual size) */
    int64_t mem_budget_bytes;
    int64_t ticks;             /* scheduler ticks run */
    int64_t admitted;          /* requests admitted so far */
    int64_t completed;         /* requests finished so far: done, failed or cancelled */
    int64_t epochs;            /* SVREM epochs run so far, over all requests */
    int64_t cached_bytes;      /* device memory kept for later admissions: blocks of finished
                                  requests and matrices no resident request uses
                                  (used_bytes + cached_bytes stays within the budget; freed by
                                  svr_serve_destroy or when an admission needs the room) */
    int64_t block_reuses;      /* allocations served from those kept blocks so far */
    int64_t matrix_reuses;     /* admissions that used a matrix already built (share_matrices) */
} svr_serve_stats_t;
/* Errors: SVR_EINVAL (NULL argument). */
int  svr_serve_stats(const svr_server *S, svr_serve_stats_t *out);
/* Gives back device memory the server keeps for later admissions: with
 * drop_matrices = 1 every idle matrix (a later request of its key builds it
 * again; its blocks join the kept blocks), then kept blocks beyond keep_bytes
 * (freed stream-ordered).  Memory of resident requests is untouched.
 * Errors: SVR_EINVAL (NULL server, drop_matrices not 0/1, keep_bytes < 0). */
int  svr_serve_trim(svr_server *S, int32_t drop_matrices, int64_t keep_bytes);

#ifdef __cplusplus
}
#endif
#endif /* SVR_H */
