// Slice stacks: S images that share one 2D system matrix, processed as one
// sparse-times-dense product per subset (slices as columns).
//
// Layout: images X[n][s], data and ratios [row][s] (subset-ordered rows), so
// a matrix entry multiplies one contiguous run of S values.  A wavefront
// covers 64 slices of one row (forward) or one transposed row (back-
// projection): it loads 64 index/weight entries with one coalesced load,
// broadcasts them one at a time with readlane, and every broadcast entry
// drives one coalesced 256-byte gather over the slices.  The matrix is read
// once per row for all slices; products and sums are FP64 in entry order.
//
// The per-(pixel, slice) OSEM and SVREM math is the single-slice one
// (phases.h); the penalty adds the two axial neighbours when asked.
#include <cmath>

#include "common.h"
#include "kernels.h"
#include "penalty.h"
#include "phases.h"

namespace svr {

constexpr int MS_THREADS = 256;
constexpr int MS_WAVES = MS_THREADS / 64;
constexpr int MS_U = 8;

__device__ inline int rl_i(int v, int j) { return __builtin_amdgcn_readlane(v, j); }
__device__ inline float rl_f(float v, int j) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j)); }

// sum over the entries [beg, end) of idx/val of val * y[idx*S + s]; wave-uniform
// beg/end; lanes with act = false load nothing and return 0
template <typename WT, typename IT>
__device__ inline double ms_dot(const IT *__restrict__ idx, const WT *__restrict__ val, int beg, int end,
                                const float *__restrict__ y, int S, int s, bool act, int lane) {
    // loads are unconditional (padded index/weight arrays, slice 0 for lanes
    // past the stack) so a batch's gathers are in flight together; entries
    // past the row and inactive lanes are masked out of the sum
    double acc = 0.0;
    const int sc = act ? s : 0;
    for (int base = beg; base < end; base += 64) {
        const int i = base + lane;
        const int ci = (int)idx[i];
        const float ai = load_w(val[i]);
        const int cv = i < end ? ci : 0;
        const int cnt = min(64, end - base);
        for (int j = 0; j < cnt; j += MS_U) {
            float x[MS_U], a[MS_U];
#pragma unroll
            for (int u = 0; u < MS_U; ++u) {
                const int c = rl_i(cv, (j + u) & 63);
                a[u] = rl_f(ai, (j + u) & 63);
                x[u] = y[(int64_t)c * S + sc];
            }
#pragma unroll
            for (int u = 0; u < MS_U; ++u)
                if (j + u < cnt) acc = acc + (double)a[u] * (double)x[u];
        }
    }
    return act ? acc : 0.0;
}

// ---- penalty with in-plane and optional axial neighbours ---------------------
// (all neighbour values loaded first, absent ones clamped in bounds and
// skipped, so the sums are those of the in-plane order then down, up)
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
        const double d = w * pot_gamma(p.potential, fn - fj, p.delta);
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

// ---- forward: MODE 1 ratio, MODE 2 log-likelihood partials -------------------
template <int MODE, typename WT, typename IT>
__global__ void __launch_bounds__(MS_THREADS)
k_ms_forward(const int *__restrict__ row_ptr, const IT *__restrict__ col, const WT *__restrict__ val, int r0,
             int r1, int S, int nch, const float *__restrict__ X, const float *__restrict__ g,
             const float *__restrict__ w, float *__restrict__ ratio, double *__restrict__ part, int *bad) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t task = (int64_t)blockIdx.x * MS_WAVES + wv;
    const int r = r0 + (int)(task / nch), c = (int)(task % nch);
    const bool valid = r < r1;
    const int s = c * 64 + lane;
    const bool act = valid && s < S;
    double acc = 0.0;
    if (valid) acc = ms_dot(col, val, row_ptr[r], row_ptr[r + 1], X, S, s, act, lane);
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

// ---- fused back-projection + OSEM / SVREM update -----------------------------
template <int KIND, typename WT, typename IT>
__global__ void __launch_bounds__(MS_THREADS)
k_ms_update(const int *__restrict__ ptrT, const IT *__restrict__ rowT, const WT *__restrict__ valT,
            const float *__restrict__ sens_t, const double *__restrict__ sens, int N, int S, int nch, int axial,
            UpdateArgs u) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t task = (int64_t)blockIdx.x * MS_WAVES + wv;
    const int n = (int)(task / nch), c = (int)(task % nch);
    const bool valid = n < N;
    const int s = c * 64 + lane;
    const bool act = valid && s < S;
    const int64_t q = (int64_t)u.t * N + n;
    const int64_t i = (int64_t)n * S + s;
    const PenaltyArgs &p = u.pen;
    float f = 0.0f, st = 0.0f, tab = 0.0f;
    double sh0 = 0.0, sanc = 0.0, sn = 0.0, D = 0.0, E = 0.0;
    if (act) {
        f = u.f[i];
        if (KIND == UPD_OSEM) {
            st = sens_t[q];
        } else {
            sh0 = u.s_hat[i];
            tab = u.table[q * S + s];
            sanc = u.s_anc[i];
            sn = sens[n];
            if (p.beta > 0.0) surrogate_at_ms(u.f, n, s, S, p, axial, D, E);
        }
    }
    double b = 0.0;
    if (valid) b = ms_dot(rowT, valT, ptrT[q], ptrT[q + 1], u.ratio, S, s, act, lane);
    if (!act) return;
    if (KIND == UPD_OSEM) {
        u.f_out[i] = osem_math(f, b, st);
    } else {
        double sh;
        u.f_out[i] = svrem_math(u.Ns, u.alpha, p.beta, f, b, sh0, tab, sanc, sn, D, E, &sh);
        u.s_hat[i] = sh;
    }
}

// ---- SVREM anchor: tau table and FP64 sums -----------------------------------
template <typename WT, typename IT>
__global__ void __launch_bounds__(MS_THREADS)
k_ms_anchor_table(const int *__restrict__ ptrT, const IT *__restrict__ rowT, const WT *__restrict__ valT,
                  const int *__restrict__ row_start, int Ns, int N, int S, int nch, const float *__restrict__ ratio,
                  const float *__restrict__ X, float *__restrict__ table) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t task = (int64_t)blockIdx.x * MS_WAVES + wv;
    const int64_t q = task / nch;
    const int c = (int)(task % nch);
    const bool valid = q < (int64_t)Ns * N;
    const int s = c * 64 + lane;
    const bool act = valid && s < S;
    if (!valid) return;  // wave-uniform
    const int t = (int)(q / N), n = (int)(q - (int64_t)t * N);
    const float f = act ? X[(int64_t)n * S + s] : 0.0f;
    const double b = ms_dot(rowT, valT, ptrT[q], ptrT[q + 1], ratio + (int64_t)row_start[t] * S, S, s, act, lane);
    if (act) table[q * S + s] = tau_of(Ns, f, b);
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

int ms_forward(const Matrix &A, int r0, int r1, int mode, int S, const float *X, const float *g, const float *w,
               float *ratio, double *part, int *bad, hipStream_t s, int *nb_out) {
    const int nch = nchunks(S);
    const unsigned nb = blocks_for((int64_t)(r1 - r0) * nch);
    if (nb_out) *nb_out = (int)nb;
    if (nb == 0) return SVR_OK;
    return with_types(A, [&](auto wv, auto iv) {
        using WT = decltype(wv);
        using IT = decltype(iv);
        if (mode == 1)
            SVR_HIP(launch_k(k_ms_forward<1, WT, IT>, nb, MS_THREADS, s, A.d_row_ptr, (const IT *)A.d_col,
                             (const WT *)A.d_val, r0, r1, S, nch, X, g, w, ratio, part, bad));
        else
            SVR_HIP(launch_k(k_ms_forward<2, WT, IT>, nb, MS_THREADS, s, A.d_row_ptr, (const IT *)A.d_col,
                             (const WT *)A.d_val, r0, r1, S, nch, X, g, w, ratio, part, bad));
        return SVR_OK;
    });
}

int ms_update(const Matrix &A, int kind, int S, int axial, const UpdateArgs &u, hipStream_t s) {
    const int nch = nchunks(S);
    const unsigned nb = blocks_for((int64_t)A.N * nch);
    if (kind != UPD_OSEM && kind != UPD_SVREM) {
        set_error("slice stacks support OSEM and SVREM updates");
        return SVR_EINVAL;
    }
    return with_types(A, [&](auto wv, auto iv) {
        using WT = decltype(wv);
        using IT = decltype(iv);
        if (kind == UPD_OSEM)
            SVR_HIP(launch_k(k_ms_update<UPD_OSEM, WT, IT>, nb, MS_THREADS, s, A.d_ptrT, (const IT *)A.d_rowT,
                             (const WT *)A.d_valT, A.d_sens_t, A.d_sens, A.N, S, nch, axial, u));
        else
            SVR_HIP(launch_k(k_ms_update<UPD_SVREM, WT, IT>, nb, MS_THREADS, s, A.d_ptrT, (const IT *)A.d_rowT,
                             (const WT *)A.d_valT, A.d_sens_t, A.d_sens, A.N, S, nch, axial, u));
        return SVR_OK;
    });
}

int ms_anchor_table(const Matrix &A, int S, const float *ratio_all, const float *X, float *table, hipStream_t s) {
    const int nch = nchunks(S);
    const unsigned nb = blocks_for((int64_t)A.Ns * A.N * nch);
    return with_types(A, [&](auto wv, auto iv) {
        using WT = decltype(wv);
        using IT = decltype(iv);
        SVR_HIP(launch_k(k_ms_anchor_table<WT, IT>, nb, MS_THREADS, s, A.d_ptrT, (const IT *)A.d_rowT,
                         (const WT *)A.d_valT, A.d_row_start, A.Ns, A.N, S, nch, ratio_all, X, table));
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
