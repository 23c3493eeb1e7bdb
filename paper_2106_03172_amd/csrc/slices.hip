// Slice stacks: S images that share one 2D system matrix, processed as one
// sparse-times-dense product per subset (slices as columns).
//
// Layout: images X[n][s], data and ratios [row][s] (subset-ordered rows), so
// a matrix entry multiplies one contiguous run of S values.  A wavefront
// covers 64 slices of one row segment (forward) or one transposed row (back-
// projection): it walks the entries with scalar loads, and every entry drives
// one coalesced 256-byte gather over the slices (ms_dot).  Products and sums
// are FP64 in entry order.
//
// The stack (41 MB at 127 x 285^2) does not fit an XCD's 4 MB L2, and every
// view's rays sweep the whole image, so gathers in row order miss the L2 and
// stream the stack from the Infinity Cache again for every view.  The passes
// therefore work region by region (StackPlan, common.h): XCD x handles the
// image regions q = x (mod XCDS) one after another, so the gathers of a pass
// hit the L2 that holds the region's slab of the stack.
//  - forward: a wavefront sums one segment of a row (the entries inside one
//    region) into an FP64 partial; a second kernel adds each row's partials
//    in ray order and forms the ratio (or the log-likelihood term);
//  - back-projection (update, anchor table): a wavefront takes one pixel of
//    the XCD's regions; the rays crossing a region touch a small part of the
//    subset's ratio block, which stays in L2.  Which wavefront takes a pixel
//    changes nothing in its arithmetic.
//
// The per-(pixel, slice) OSEM and SVREM math is the single-slice one
// (phases.h); the penalty adds the two axial neighbours when asked.
#include <cmath>

#include "common.h"
#include "kernels.h"
#include "penalty.h"
#include "phases.h"
#include "util.h"

namespace svr {

constexpr int MS_THREADS = 256;
constexpr int MS_WAVES = MS_THREADS / 64;
constexpr int MS_U = 8;

// For c < NC: acc[c] = sum over the entries [beg, end) of idx/val of
// val * y[idx*S + s0 + 64c]; beg/end wave-uniform; slices at or past S load
// slice 0 and give 0.
//
// The entry index walks the row wave-uniformly, so every index and weight is
// one scalar load shared by the wavefront (no cross-lane moves) and serves all
// NC chunks, and each gather is a buffer load whose per-entry offset idx*S*4
// sits in an SGPR, the lane's own slice offset in a loop-invariant VGPR.  What
// is left per entry and chunk on the vector unit is the two conversions to
// FP64 and one FMA (the product of two FP32 values is exact in FP64, so the FMA
// rounds like a multiply followed by an add).  Every slice adds its entries in
// row order.
template <int NC, typename WT, typename IT>
__device__ inline void ms_dot(const IT *__restrict__ idx, const WT *__restrict__ val, int beg, int end,
                              const float *__restrict__ y, int S, int s0, double (&acc)[NC]) {
    const __amdgpu_buffer_rsrc_t ry = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(y), (short)0,
                                                                        0x7fffffff, BUF_RSRC_WORD3);
    int vo[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        vo[c] = (s0 + 64 * c < S ? s0 + 64 * c : 0) * 4;
        acc[c] = 0.0;
    }
    const int row_bytes = S * 4;
    int i = beg;
    // software-pipelined: the next batch's indices and weights are loaded
    // while the current batch's gathers are in flight
    int cn[MS_U];
    float an[MS_U];
    bool more = i + MS_U <= end;
    if (more) {
#pragma unroll
        for (int u = 0; u < MS_U; ++u) {
            cn[u] = (int)idx[i + u];
            an[u] = load_w(val[i + u]);
        }
    }
    while (more) {
        float x[MS_U][NC], a[MS_U];
#pragma unroll
        for (int u = 0; u < MS_U; ++u) {
            const int off = cn[u] * row_bytes;
            a[u] = an[u];
#pragma unroll
            for (int c = 0; c < NC; ++c)
                x[u][c] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ry, vo[c], off, 0));
        }
        i += MS_U;
        more = i + MS_U <= end;
        if (more) {
#pragma unroll
            for (int u = 0; u < MS_U; ++u) {
                cn[u] = (int)idx[i + u];
                an[u] = load_w(val[i + u]);
            }
        }
#pragma unroll
        for (int u = 0; u < MS_U; ++u) {
            const double ad = (double)a[u];
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c] = __builtin_fma(ad, (double)x[u][c], acc[c]);
        }
    }
    for (; i < end; ++i) {
        const int off = (int)idx[i] * row_bytes;
        const double ad = (double)load_w(val[i]);
#pragma unroll
        for (int c = 0; c < NC; ++c)
            acc[c] = __builtin_fma(ad, (double)__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ry, vo[c], off, 0)),
                                   acc[c]);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (s0 + 64 * c >= S) acc[c] = 0.0;
}

// ---- penalty with in-plane and optional axial neighbours ---------------------
// (all neighbour values loaded first, absent ones clamped in bounds and
// skipped, so the sums are those of the in-plane order then down, up)
template <int POT>
__device__ inline void surrogate_at_ms(const float *X, int n, int s, int S, const PenaltyArgs &p, int axial,
                                       double &D, double &E) {
    const int iy = n / p.nx, ix = n - iy * p.nx;
    const double fn = (double)X[(int64_t)n * S + s];
    const Neighbours nb = load_neighbours(X, ix, iy, p.nx, p.ny, S, s);
    const double fd = (double)X[(int64_t)n * S + (s > 0 ? s - 1 : s)];
    const double fu = (double)X[(int64_t)n * S + (s + 1 < S ? s + 1 : s)];
    D = 0.0;
    E = 0.0;
    auto add = [&](double fj, double w) {
        const double d = w * pot_gamma(POT, fn - fj, p.delta);
        D = D + d;
        E = E + d * fj;
    };
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (nb.ok[k]) add((double)nb.v[k], nb_weight(k));
    if (axial) {
        if (s > 0) add(fd, 1.0);
        if (s + 1 < S) add(fu, 1.0);
    }
}

__device__ inline double penalty_share_at_ms(const float *X, int n, int s, int S, const PenaltyArgs &p, int axial) {
    const int iy = n / p.nx, ix = n - iy * p.nx;
    const double fn = (double)X[(int64_t)n * S + s];
    const Neighbours nb = load_neighbours(X, ix, iy, p.nx, p.ny, S, s);
    const double fd = (double)X[(int64_t)n * S + (s > 0 ? s - 1 : s)];
    const double fu = (double)X[(int64_t)n * S + (s + 1 < S ? s + 1 : s)];
    double r = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (nb.ok[k]) r = r + nb_weight(k) * pot_rho(p.potential, fn - (double)nb.v[k], p.delta);
    if (axial) {
        if (s > 0) r = r + pot_rho(p.potential, fn - fd, p.delta);
        if (s + 1 < S) r = r + pot_rho(p.potential, fn - fu, p.delta);
    }
    return 0.5 * r;
}

// ---- regions ------------------------------------------------------------------
__host__ __device__ inline int region_of_pixel(int n, int nx, const Regions &g) {
    const int iy = n / nx, ix = n - iy * nx;
    return (iy / g.ly) * g.rx + ix / g.lx;
}

// Pixel p (0-based) of the regions of XCD x, region-major (q = x, x + XCDS,
// ...), row-major inside a region; -1 past the last.  Wave-uniform inputs.
__device__ inline int region_pixel(const Regions &g, int x, int p, int nx, int ny) {
    for (int q = x; q < g.ry * g.rx; q += XCDS) {
        const int qy = q / g.rx;
        const int y0 = qy * g.ly, x0 = (q - qy * g.rx) * g.lx;
        const int h = min(g.ly, ny - y0), w = min(g.lx, nx - x0);
        if (h <= 0 || w <= 0) continue;
        const int a = h * w;
        if (p < a) {
            const int py = p / w;
            return (y0 + py) * nx + x0 + (p - py * w);
        }
        p -= a;
    }
    return -1;
}

// ---- forward: segment sums, then per-row sums ----------------------------------
// Slices are taken in groups of NC chunks of 64 (ng = ceil(nch / NC) groups).
// Task p of XCD x in a schedule: segment sched[off[x] + p / ng], group p mod ng.
// P[k][s] = sum over segment k's entries of a * X[n][s].
template <int NC, typename WT, typename IT>
__global__ void __launch_bounds__(MS_THREADS)
k_ms_seg_dot(const IT *__restrict__ col, const WT *__restrict__ val, const int *__restrict__ seg_beg,
             const int *__restrict__ sched, XcdSched xs, int S, int nch, int ng, const float *__restrict__ X,
             double *__restrict__ P) {
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int x = blockIdx.x % XCDS;
    const int p = (int)(blockIdx.x / XCDS) * MS_WAVES + wv;
    if (p >= xs.cnt[x] * ng) return;  // wave-uniform
    const int item = p / ng, grp = p - item * ng;
    const int k = __builtin_amdgcn_readfirstlane(sched[xs.off[x] + item]);
    const int beg = __builtin_amdgcn_readfirstlane(seg_beg[k]);
    const int end = __builtin_amdgcn_readfirstlane(seg_beg[k + 1]);
    const int s0 = grp * NC * 64 + lane;
    double acc[NC];
    ms_dot<NC>(col, val, beg, end, X, S, s0, acc);
    double *Pk = P + (int64_t)k * (nch * 64);
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (s0 + 64 * c < nch * 64) Pk[s0 + 64 * c] = acc[c];  // slices past S write 0 into the padding
}

// Row r's sums: its segments' partials in ray order.  MODE 1 writes the
// ratios, MODE 2 the log-likelihood partials of the block (summed afterwards
// in a fixed order).  One wavefront per (row, chunk of 64 slices).
template <int MODE>
__global__ void __launch_bounds__(MS_THREADS)
k_ms_seg_rows(const int *__restrict__ seg_ptr, int r0, int r1, int S, int nch, const double *__restrict__ P,
              const float *__restrict__ g, const float *__restrict__ w, float *__restrict__ ratio,
              double *__restrict__ part, int *bad) {
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int task = (int)blockIdx.x * MS_WAVES + wv;
    const int rr = task / nch, c = task - rr * nch;
    const int r = r0 + rr;
    const bool valid = r < r1;
    const int s = c * 64 + lane;
    const bool act = valid && s < S;
    double acc = 0.0;
    if (valid) {
        const int kb = __builtin_amdgcn_readfirstlane(seg_ptr[r]), ke = __builtin_amdgcn_readfirstlane(seg_ptr[r + 1]);
        const double *Pc = P + s;
        const int64_t ld = (int64_t)nch * 64;
        int k = kb;
        for (; k + 4 <= ke; k += 4) {  // four independent loads, added in order
            const double a0 = Pc[(int64_t)k * ld], a1 = Pc[(int64_t)(k + 1) * ld];
            const double a2 = Pc[(int64_t)(k + 2) * ld], a3 = Pc[(int64_t)(k + 3) * ld];
            acc = acc + a0;
            acc = acc + a1;
            acc = acc + a2;
            acc = acc + a3;
        }
        for (; k < ke; ++k) acc = acc + Pc[(int64_t)k * ld];
    }
    const int64_t i = (int64_t)r * S + s;
    if (MODE == 1) {
        if (act) ratio[i] = em_ratio(g[i], acc + (double)w[i]);
    } else {
        __shared__ double wsum[MS_WAVES];
        double term = 0.0;
        if (act) {
            const double yb = acc + (double)w[i];
            const float gv = g[i];
            if (gv > 0.0f) {
                if (yb > 0.0) term = (double)gv * log(yb) - yb;
                else atomicOr(bad, 1);
            } else {
                term = -yb;
            }
        }
        term = wave_sum(term);
        if (lane == 0) wsum[wv] = term;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int k = 0; k < MS_WAVES; ++k) t = t + wsum[k];
            part[blockIdx.x] = t;
        }
    }
}

// ---- plan: segments and schedules ------------------------------------------------
template <typename IT>
__global__ void k_seg_count(const int *__restrict__ row_ptr, const IT *__restrict__ col, int M, int nx, Regions g,
                            int *__restrict__ cnt) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= M) return;
    int c = 0, prev = -1;
    for (int i = row_ptr[r]; i < row_ptr[r + 1]; ++i) {
        const int q = region_of_pixel((int)col[i], nx, g);
        c += q != prev;
        prev = q;
    }
    cnt[r] = c;
}

template <typename IT>
__global__ void k_seg_fill(const int *__restrict__ row_ptr, const IT *__restrict__ col, int M, int nx, Regions g,
                           const int *__restrict__ seg_ptr, int *__restrict__ seg_beg, int *__restrict__ seg_q) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= M) return;
    int k = seg_ptr[r], prev = -1;
    for (int i = row_ptr[r]; i < row_ptr[r + 1]; ++i) {
        const int q = region_of_pixel((int)col[i], nx, g);
        if (q != prev) {
            seg_beg[k] = i;
            seg_q[k] = q;
            ++k;
        }
        prev = q;
    }
}

// ---- fused back-projection + OSEM / SVREM update -----------------------------
// task p of XCD x: pixel region_pixel(x, p / ng), slice group p mod ng
template <int KIND, int NC, typename WT, typename IT, int POT>
__global__ void __launch_bounds__(MS_THREADS)
k_ms_update(const int *__restrict__ ptrT, const IT *__restrict__ rowT, const WT *__restrict__ valT,
            const float *__restrict__ sens_t, const double *__restrict__ sens, int N, int S, int ng, int axial,
            Regions rg, UpdateArgs u) {
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int x = blockIdx.x % XCDS;
    const int task = (int)(blockIdx.x / XCDS) * MS_WAVES + wv;
    const int item = task / ng, grp = task - item * ng;
    const int n = region_pixel(rg, x, item, u.pen.nx, u.pen.ny);
    if (n < 0) return;  // wave-uniform
    const int64_t q = (int64_t)u.t * N + n;
    const int s0 = grp * NC * 64 + lane;
    const PenaltyArgs &p = u.pen;
    float f[NC], tab[NC];
    double sh0[NC], sanc[NC], D[NC], E[NC];
    float st = 0.0f;
    double sn = 0.0;
    if (KIND == UPD_OSEM) st = sens_t[q];
    else sn = sens[n];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int s = s0 + 64 * c;
        const int64_t i = (int64_t)n * S + s;
        f[c] = tab[c] = 0.0f;
        sh0[c] = sanc[c] = D[c] = E[c] = 0.0;
        if (s < S) {
            f[c] = u.f[i];
            if (KIND != UPD_OSEM) {
                sh0[c] = u.s_hat[i];
                tab[c] = u.table[q * S + s];
                sanc[c] = u.s_anc[i];
                if (p.beta > 0.0) surrogate_at_ms<POT>(u.f, n, s, S, p, axial, D[c], E[c]);
            }
        }
    }
    const int beg = __builtin_amdgcn_readfirstlane(ptrT[q]), end = __builtin_amdgcn_readfirstlane(ptrT[q + 1]);
    double b[NC];
    ms_dot<NC>(rowT, valT, beg, end, u.ratio, S, s0, b);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int s = s0 + 64 * c;
        if (s >= S) continue;
        const int64_t i = (int64_t)n * S + s;
        if (KIND == UPD_OSEM) {
            u.f_out[i] = osem_math(f[c], b[c], st);
        } else {
            double sh;
            u.f_out[i] = svrem_math(u.Ns, u.alpha, p.beta, f[c], b[c], sh0[c], tab[c], sanc[c], sn, D[c], E[c], &sh);
            u.s_hat[i] = sh;
        }
    }
}

// ---- SVREM anchor: tau table and FP64 sums -----------------------------------
// Task p of XCD x, region-major: the XCD's regions q = x, x + XCDS, ... in
// turn, and within a region every subset t, then the region's pixels
// (row-major), then the slice group.  A region's slab of the stack stays in
// the L2 while all subsets visit it (tau_t reads f for every t), and each
// subset's ratios of the rays crossing the region are streamed once.
template <int NC, typename WT, typename IT>
__global__ void __launch_bounds__(MS_THREADS)
k_ms_anchor_table(const int *__restrict__ ptrT, const IT *__restrict__ rowT, const WT *__restrict__ valT,
                  const int *__restrict__ row_start, int Ns, int N, int S, int ng, int nx, int ny, Regions rg,
                  const float *__restrict__ ratio, const float *__restrict__ X, float *__restrict__ table) {
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int x = blockIdx.x % XCDS;
    int p = (int)(blockIdx.x / XCDS) * MS_WAVES + wv;
    int n = -1, t = 0, grp = 0;
    for (int q = x; q < rg.ry * rg.rx; q += XCDS) {  // wave-uniform walk over the XCD's regions
        const int qy = q / rg.rx;
        const int y0 = qy * rg.ly, x0 = (q - qy * rg.rx) * rg.lx;
        const int h = min(rg.ly, ny - y0), w = min(rg.lx, nx - x0);
        if (h <= 0 || w <= 0) continue;
        const int per_t = h * w * ng;
        if (p < per_t * Ns) {
            t = p / per_t;
            const int rem = p - t * per_t;
            const int item = rem / ng;
            grp = rem - item * ng;
            const int py = item / w;
            n = (y0 + py) * nx + x0 + (item - py * w);
            break;
        }
        p -= per_t * Ns;
    }
    if (n < 0) return;  // wave-uniform
    const int64_t q = (int64_t)t * N + n;
    const int s0 = grp * NC * 64 + lane;
    float f[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) f[c] = s0 + 64 * c < S ? X[(int64_t)n * S + s0 + 64 * c] : 0.0f;
    const int beg = __builtin_amdgcn_readfirstlane(ptrT[q]), end = __builtin_amdgcn_readfirstlane(ptrT[q + 1]);
    double b[NC];
    ms_dot<NC>(rowT, valT, beg, end, ratio + (int64_t)row_start[t] * S, S, s0, b);
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (s0 + 64 * c < S) table[q * S + s0 + 64 * c] = tau_of(Ns, f[c], b[c]);
}

__global__ void __launch_bounds__(256)
k_ms_anchor_sum(int Ns, int64_t NS, const float *__restrict__ table, double *__restrict__ s_anc,
                double *__restrict__ s_hat, int init_shat) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= NS) return;
    const double sum = subset_sum(table, Ns, NS, i);
    const double sa = sum / (double)Ns;
    s_anc[i] = sa;
    if (init_shat) s_hat[i] = sa;
}

__global__ void __launch_bounds__(256)
k_ms_penalty_value(const float *X, int N, int S, PenaltyArgs p, int axial, double *part) {
    __shared__ double red[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    red[threadIdx.x] = (i < (int64_t)N * S) ? penalty_share_at_ms(X, (int)(i / S), (int)(i % S), S, p, axial) : 0.0;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ---- layout conversions ------------------------------------------------------
// API sinogram [S][M] (natural rows) -> internal [subset-ordered row][S]
__global__ void k_ms_pack_sino(const int *row_sino, int M, int S, const float *src, float *dst) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)M * S) return;
    const int r = (int)(i / S), s = (int)(i % S);
    dst[i] = src[(int64_t)s * M + row_sino[r]];
}
// API image [S][N] <-> internal [N][S]
__global__ void k_ms_pack_img(int N, int S, const float *src, float *dst) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)N * S) return;
    const int n = (int)(i / S), s = (int)(i % S);
    dst[i] = src[(int64_t)s * N + n];
}
__global__ void k_ms_unpack_img(int N, int S, const float *src, float *dst) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)N * S) return;
    const int n = (int)(i / S), s = (int)(i % S);
    dst[(int64_t)s * N + n] = src[i];
}

// ---- launchers ---------------------------------------------------------------
static inline int nchunks(int S) { return (S + 63) / 64; }
static inline unsigned blocks_for(int64_t tasks) { return (unsigned)((tasks + MS_WAVES - 1) / MS_WAVES); }

static inline unsigned xcd_blocks(int64_t tasks_per_xcd) {
    return (unsigned)(XCDS * ((tasks_per_xcd + MS_WAVES - 1) / MS_WAVES));
}

Regions choose_regions(int nx, int ny, int S) {
    // the smallest grid (a multiple of XCDS regions) whose region slab of the
    // stack takes at most 2.75 MB, leaving room in the 4 MB L2 for the streams
    static const int grid[][2] = {{2, 4}, {4, 4}, {4, 8}, {8, 8}, {8, 16}, {16, 16}};
    Regions g;
    for (const auto &gr : grid) {
        g.ry = std::min(gr[0], ny);
        g.rx = std::min(gr[1], nx);
        g.ly = (ny + g.ry - 1) / g.ry;
        g.lx = (nx + g.rx - 1) / g.rx;
        g.ry = (ny + g.ly - 1) / g.ly;  // no empty regions
        g.rx = (nx + g.lx - 1) / g.lx;
        if ((double)g.ly * g.lx * S * 4.0 <= 2.75e6) break;
    }
    return g;
}

void ms_plan_free(StackPlan &plan) {
    dfree(plan.seg_ptr);
    dfree(plan.seg_beg);
    dfree(plan.sched_sub);
    dfree(plan.sched_all);
    dfree(plan.P);
    plan = StackPlan{};
}

int ms_plan_build(const Matrix &A, int S, StackPlan &plan, hipStream_t s) {
    const int M = A.M, nx = A.geom.nx, ny = A.geom.ny;
    plan.S = S;
    plan.nch = nchunks(S);
    plan.reg = choose_regions(nx, ny, S);
    const Regions g = plan.reg;
    const int Q = g.ry * g.rx;
    int *cnt = nullptr, *seg_q = nullptr;
    auto fail = [&](int rc) {
        dfree(cnt);
        dfree(seg_q);
        ms_plan_free(plan);
        return rc;
    };
    if (dalloc(&cnt, M) != hipSuccess || dalloc(&plan.seg_ptr, M + 1) != hipSuccess) {
        set_error("no device memory for the stack plan");
        return fail(SVR_ENOMEM);
    }
    const unsigned gm = (unsigned)((M + 255) / 256);
    int rc = with_types(A, [&](auto, auto iv) {
        using IT = decltype(iv);
        k_seg_count<IT><<<gm, 256, 0, s>>>(A.d_row_ptr, (const IT *)A.d_col, M, nx, g, cnt);
        SVR_HIP(hipGetLastError());
        return SVR_OK;
    });
    if (rc) return fail(rc);
    int64_t nseg = 0;
    rc = exclusive_scan(cnt, M, plan.seg_ptr, &nseg, s);  // synchronises
    if (rc) return fail(rc);
    plan.nseg = nseg;
    if (dalloc(&plan.seg_beg, nseg + 1) != hipSuccess || dalloc(&seg_q, std::max<int64_t>(nseg, 1)) != hipSuccess ||
        dalloc(&plan.sched_sub, std::max<int64_t>(nseg, 1)) != hipSuccess ||
        dalloc(&plan.sched_all, std::max<int64_t>(nseg, 1)) != hipSuccess ||
        dalloc(&plan.P, std::max<int64_t>(nseg, 1) * plan.nch * 64) != hipSuccess) {
        set_error("no device memory for the stack plan (%lld segments)", (long long)nseg);
        return fail(SVR_ENOMEM);
    }
    rc = with_types(A, [&](auto, auto iv) {
        using IT = decltype(iv);
        k_seg_fill<IT><<<gm, 256, 0, s>>>(A.d_row_ptr, (const IT *)A.d_col, M, nx, g, plan.seg_ptr, plan.seg_beg,
                                         seg_q);
        SVR_HIP(hipGetLastError());
        return SVR_OK;
    });
    if (rc) return fail(rc);
    const int nnz32 = (int)A.nnz;
    SVR_HIP(hipMemcpyAsync(plan.seg_beg + nseg, &nnz32, sizeof(int), hipMemcpyHostToDevice, s));
    // schedules on the host: segments grouped by XCD, region-major, in segment order
    std::vector<int> hq(nseg), hptr(M + 1);
    SVR_HIP(hipMemcpyAsync(hq.data(), seg_q, sizeof(int) * nseg, hipMemcpyDeviceToHost, s));
    SVR_HIP(hipMemcpyAsync(hptr.data(), plan.seg_ptr, sizeof(int) * (M + 1), hipMemcpyDeviceToHost, s));
    SVR_HIP(hipStreamSynchronize(s));
    dfree(seg_q);
    seg_q = nullptr;
    dfree(cnt);
    cnt = nullptr;
    std::vector<int> sub(nseg), all(nseg);
    auto group = [&](int64_t k0, int64_t k1, int *dst, XcdSched &xs, int base) {
        std::vector<std::vector<int>> byq(Q);
        for (int64_t k = k0; k < k1; ++k) byq[hq[k]].push_back((int)k);
        int pos = base;
        for (int x = 0; x < XCDS; ++x) {
            xs.off[x] = pos;
            for (int q = x; q < Q; q += XCDS)
                for (int k : byq[q]) dst[pos++] = k;
            xs.cnt[x] = pos - xs.off[x];
        }
        return pos;
    };
    plan.sub.assign(A.Ns, XcdSched{});
    int pos = 0;
    for (int t = 0; t < A.Ns; ++t)
        pos = group(hptr[A.row_start[t]], hptr[A.row_start[t + 1]], sub.data(), plan.sub[t], pos);
    group(0, nseg, all.data(), plan.all, 0);
    if (nseg > 0) {
        SVR_HIP(hipMemcpyAsync(plan.sched_sub, sub.data(), sizeof(int) * nseg, hipMemcpyHostToDevice, s));
        SVR_HIP(hipMemcpyAsync(plan.sched_all, all.data(), sizeof(int) * nseg, hipMemcpyHostToDevice, s));
    }
    for (int x = 0; x < XCDS; ++x) plan.area[x] = 0;
    for (int q = 0; q < Q; ++q) {
        const int y0 = (q / g.rx) * g.ly, x0 = (q % g.rx) * g.lx;
        plan.area[q % XCDS] += std::max(0, std::min(g.ly, ny - y0)) * std::max(0, std::min(g.lx, nx - x0));
    }
    SVR_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
    return SVR_OK;
}

int ms_forward(const Matrix &A, const StackPlan &plan, int t, int mode, int S, const float *X, const float *g,
               const float *w, float *ratio, double *part, int *bad, hipStream_t s, int *nb_out) {
    const int nch = nchunks(S);
    const int r0 = t < 0 ? 0 : A.row_start[t], r1 = t < 0 ? A.M : A.row_start[t + 1];
    const XcdSched &xs = t < 0 ? plan.all : plan.sub[t];
    const int *sched = t < 0 ? plan.sched_all : plan.sched_sub;
    const int nc = nch > 1 ? 2 : 1, ng = (nch + nc - 1) / nc;
    int most = 0;
    for (int x = 0; x < XCDS; ++x) most = std::max(most, xs.cnt[x]);
    const unsigned nbd = xcd_blocks((int64_t)most * ng);
    const unsigned nb = blocks_for((int64_t)(r1 - r0) * nch);
    if (nb_out) *nb_out = (int)nb;
    if (nb == 0) return SVR_OK;
    int rc = SVR_OK;
    LaunchEvents &tm = pending_timing();
    if (tm.start && nbd > 0) tm.span = 2;  // a timed forward covers both kernels
    if (nbd > 0) {
        rc = with_types(A, [&](auto wv, auto iv) {
            using WT = decltype(wv);
            using IT = decltype(iv);
            if (nc == 2)
                SVR_HIP(launch_k(k_ms_seg_dot<2, WT, IT>, nbd, MS_THREADS, s, (const IT *)A.d_col, (const WT *)A.d_val,
                                 (const int *)plan.seg_beg, sched, xs, S, nch, ng, X, plan.P));
            else
                SVR_HIP(launch_k(k_ms_seg_dot<1, WT, IT>, nbd, MS_THREADS, s, (const IT *)A.d_col, (const WT *)A.d_val,
                                 (const int *)plan.seg_beg, sched, xs, S, nch, ng, X, plan.P));
            return SVR_OK;
        });
        if (rc) return rc;
    }
    if (mode == 1)
        SVR_HIP(launch_k(k_ms_seg_rows<1>, nb, MS_THREADS, s, (const int *)plan.seg_ptr, r0, r1, S, nch,
                         (const double *)plan.P, g, w, ratio, part, bad));
    else
        SVR_HIP(launch_k(k_ms_seg_rows<2>, nb, MS_THREADS, s, (const int *)plan.seg_ptr, r0, r1, S, nch,
                         (const double *)plan.P, g, w, ratio, part, bad));
    return SVR_OK;
}

// the potential is a template argument, as in the single-slice stencil, so
// each neighbour's curvature is the potential's own expression
template <int KIND, int NC, int POT>
static int ms_update_p(const Matrix &A, const StackPlan &plan, int S, int ng, int axial, const UpdateArgs &u,
                       unsigned nb, hipStream_t s) {
    return with_types(A, [&](auto wv, auto iv) {
        using WT = decltype(wv);
        using IT = decltype(iv);
        SVR_HIP(launch_k(k_ms_update<KIND, NC, WT, IT, POT>, nb, MS_THREADS, s, A.d_ptrT, (const IT *)A.d_rowT,
                         (const WT *)A.d_valT, A.d_sens_t, A.d_sens, A.N, S, ng, axial, plan.reg, u));
        return SVR_OK;
    });
}

template <int KIND, int NC>
static int ms_update_t(const Matrix &A, const StackPlan &plan, int S, int ng, int axial, const UpdateArgs &u,
                       unsigned nb, hipStream_t s) {
    switch (u.pen.potential) {
        case SVR_PEN_HUBER: return ms_update_p<KIND, NC, SVR_PEN_HUBER>(A, plan, S, ng, axial, u, nb, s);
        case SVR_PEN_LOGCOSH: return ms_update_p<KIND, NC, SVR_PEN_LOGCOSH>(A, plan, S, ng, axial, u, nb, s);
        case SVR_PEN_HYPERBOLA: return ms_update_p<KIND, NC, SVR_PEN_HYPERBOLA>(A, plan, S, ng, axial, u, nb, s);
        default: return ms_update_p<KIND, NC, SVR_PEN_QUADRATIC>(A, plan, S, ng, axial, u, nb, s);
    }
}

int ms_update(const Matrix &A, const StackPlan &plan, int kind, int S, int axial, const UpdateArgs &u, hipStream_t s) {
    const int nch = nchunks(S);
    const int nc = nch > 1 ? 2 : 1, ng = (nch + nc - 1) / nc;
    int most = 0;
    for (int x = 0; x < XCDS; ++x) most = std::max(most, plan.area[x]);
    const unsigned nb = xcd_blocks((int64_t)most * ng);
    if (kind != UPD_OSEM && kind != UPD_SVREM) {
        set_error("slice stacks support OSEM and SVREM updates");
        return SVR_EINVAL;
    }
    if (kind == UPD_OSEM)
        return nc == 2 ? ms_update_t<UPD_OSEM, 2>(A, plan, S, ng, axial, u, nb, s)
                       : ms_update_t<UPD_OSEM, 1>(A, plan, S, ng, axial, u, nb, s);
    return nc == 2 ? ms_update_t<UPD_SVREM, 2>(A, plan, S, ng, axial, u, nb, s)
                   : ms_update_t<UPD_SVREM, 1>(A, plan, S, ng, axial, u, nb, s);
}

int ms_anchor_table(const Matrix &A, const StackPlan &plan, int S, const float *ratio_all, const float *X,
                    float *table, hipStream_t s) {
    const int nch = nchunks(S);
    const int nc = nch > 1 ? 2 : 1, ng = (nch + nc - 1) / nc;
    int most = 0;
    for (int x = 0; x < XCDS; ++x) most = std::max(most, plan.area[x]);
    const unsigned nb = xcd_blocks((int64_t)A.Ns * most * ng);
    return with_types(A, [&](auto wv, auto iv) {
        using WT = decltype(wv);
        using IT = decltype(iv);
        if (nc == 2)
            SVR_HIP(launch_k(k_ms_anchor_table<2, WT, IT>, nb, MS_THREADS, s, A.d_ptrT, (const IT *)A.d_rowT,
                             (const WT *)A.d_valT, A.d_row_start, A.Ns, A.N, S, ng, A.geom.nx, A.geom.ny, plan.reg,
                             ratio_all, X, table));
        else
            SVR_HIP(launch_k(k_ms_anchor_table<1, WT, IT>, nb, MS_THREADS, s, A.d_ptrT, (const IT *)A.d_rowT,
                             (const WT *)A.d_valT, A.d_row_start, A.Ns, A.N, S, ng, A.geom.nx, A.geom.ny, plan.reg,
                             ratio_all, X, table));
        return SVR_OK;
    });
}

int ms_anchor_sum(const Matrix &A, int S, const float *table, double *s_anc, double *s_hat, int init_shat,
                  hipStream_t s) {
    const int64_t NS = (int64_t)A.N * S;
    SVR_HIP(launch_k(k_ms_anchor_sum, (unsigned)((NS + 255) / 256), 256, s, A.Ns, NS, table, s_anc, s_hat,
                     init_shat));
    return SVR_OK;
}

int ms_penalty_value(const Matrix &A, int S, const float *X, int potential, double delta, int axial, double *part,
                     int *nb_out, hipStream_t s) {
    PenaltyArgs p{potential, delta, 0.0, A.geom.nx, A.geom.ny};
    const int64_t NS = (int64_t)A.N * S;
    const unsigned nb = (unsigned)((NS + 255) / 256);
    *nb_out = (int)nb;
    SVR_HIP(launch_k(k_ms_penalty_value, nb, 256, s, X, A.N, S, p, axial, part));
    return SVR_OK;
}

int ms_pack_sino(const Matrix &A, int S, const float *src, float *dst, hipStream_t s) {
    const int64_t n = (int64_t)A.M * S;
    SVR_HIP(launch_k(k_ms_pack_sino, (unsigned)((n + 255) / 256), 256, s, A.d_row_sino, A.M, S, src, dst));
    return SVR_OK;
}

int ms_pack_img(int N, int S, const float *src, float *dst, hipStream_t s) {
    const int64_t n = (int64_t)N * S;
    SVR_HIP(launch_k(k_ms_pack_img, (unsigned)((n + 255) / 256), 256, s, N, S, src, dst));
    return SVR_OK;
}

int ms_unpack_img(int N, int S, const float *src, float *dst, hipStream_t s) {
    const int64_t n = (int64_t)N * S;
    SVR_HIP(launch_k(k_ms_unpack_img, (unsigned)((n + 255) / 256), 256, s, N, S, src, dst));
    return SVR_OK;
}

}  // namespace svr
