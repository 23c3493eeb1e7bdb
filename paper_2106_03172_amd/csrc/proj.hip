// Projectors: forward rows of A (with the fused EM ratio or log-likelihood)
// and the gather-only transposed back-projection.
//
// Forward: one 64-lane wavefront per row of A (passes that fit in the
// wavefronts the device holds at once: the per-subset passes) or per pair of
// consecutive rows, 32 lanes per row (larger passes: the whole matrix), lanes
// striding over the row's non-zeros (coalesced, range-checked reads of the
// index and weight streams, image gathers from L2), FP64 products and a fixed
// reduction, so a row sums in the same order in every pass of its kind.
//
// Back-projection: BP_G lanes per pixel over that pixel's transposed row of
// subset t, FP64 products, fixed butterfly reduction.
//
// Passes over many more rows than the device holds wavefronts (the whole
// matrix) can give each wavefront a run of consecutive rows and pipeline them
// (fwd_run, bp_run): per row the arithmetic is the one-pair code's, so the
// results do not depend on the run length.
#include <cmath>

#include "common.h"
#include "kernels.h"
#include "penalty.h"

namespace svr {

// g log ybar - ybar of one row (0 log 0 = 0); flags g > 0 with ybar <= 0.
// With eps > 0, rows with w = 0 and ybar <= eps take the second-order
// expansion about eps (Sec. 2.3, eq. modified_LL).
__device__ inline double loglik_term(float g, float w, double yb, double eps, int *bad) {
    if (g > 0.0f) {
        if (eps > 0.0 && w == 0.0f && yb <= eps) {
            const double gd = (double)g, d = yb - eps;
            return ((gd * log(eps) - eps) + (gd / eps - 1.0) * d) - (0.5 * (gd / (eps * eps)) * d) * d;
        }
        if (yb > 0.0) return (double)g * log(yb) - yb;
        atomicOr(bad, 1);
        return 0.0;
    }
    return -yb;
}

// Row of wavefront wv of block b in a one-row-per-wavefront pass over the
// rows r0 + j*B + bin (views j < Vt, bins bin < B) when B > 0: workgroups are
// dispatched to the XCDs round-robin (b mod XCDS), and XCD x takes the bin
// band [x B / XCDS, (x + 1) B / XCDS) of every view, bin-minor.  A band's
// rays cross a ring of the image rather than all of it, so each XCD's L2
// fetches a part of the image instead of the whole.  B = 0: row r0 + b W + wv.
// Returns -1 for a wavefront with no row.
__device__ inline int band_row(int b, int wv, int r0, int r1, int B, int Vt) {
    if (B == 0) {
        const int r = r0 + b * FWD_WAVES_PER_BLOCK + wv;
        return r < r1 ? r : -1;
    }
    const int x = b % XCDS, L = b / XCDS;
    const int lo = x * B / XCDS, w = (x + 1) * B / XCDS - lo;
    const int p = L * FWD_WAVES_PER_BLOCK + wv;
    const int j = p / w;
    return j < Vt ? r0 + j * B + lo + (p - j * w) : -1;
}

// one wavefront per row r (PAIR: per pair of rows r, r + 1); mode 0 writes
// y[row_sino[r]], mode 1 the ratio, mode 2 the row's log-likelihood term to
// part[r - r0] (summed afterwards in a fixed order).  Without PAIR the row
// comes from band_row (B, Vt); a row's arithmetic does not depend on which
// wavefront takes it.
template <int MODE, bool PAIR, typename WT, typename IT, int U = FWD_U>
__global__ void __launch_bounds__(FWD_THREADS)
k_forward(const int *__restrict__ row_ptr, const IT *__restrict__ col, const WT *__restrict__ val,
          const int *__restrict__ row_sino, int r0, int r1, int B, int Vt, FwdArgs a) {
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int r = PAIR ? r0 + 2 * (blockIdx.x * FWD_WAVES_PER_BLOCK + wv) : band_row(blockIdx.x, wv, r0, r1, B, Vt);
    if (r < 0 || r >= r1) return;  // wave-uniform
    if constexpr (!PAIR) {
        if (MODE == 1) {
            fwd_ratio_row<U>(row_ptr, col, val, a.f, a.g, a.w, a.out, r, lane, a.eps);
            return;
        }
        const double acc = wave_sum(row_dot<U>(row_ptr, col, val, a.f, r, lane));
        if (lane != 0) return;
        if (MODE == 0) a.out[row_sino[r]] = (float)acc;
        else a.part[r - r0] = loglik_term(a.g[r], a.w[r], acc + (double)a.w[r], a.eps, a.bad);
        return;
    }
    if (MODE == 1) {
        fwd_ratio_pair(row_ptr, col, val, a.f, a.g, a.w, a.out, r, r1, lane, a.eps);
        return;
    }
    const int ru = __builtin_amdgcn_readfirstlane(r);
    const int b0 = row_ptr[ru], e0 = row_ptr[ru + 1], e1 = row_ptr[min(ru + 2, r1)];
    double s0, s1;
    half_sums(pair_dot(col, val, a.f, b0, e0, e1, lane), s0, s1);
    const int h = lane >> 5, rh = ru + h;
    if ((lane & 31) != 0 || rh >= r1) return;
    const double acc = h ? s1 : s0;
    if (MODE == 0) a.out[row_sino[rh]] = (float)acc;
    else a.part[rh - r0] = loglik_term(a.g[rh], a.w[rh], acc + (double)a.w[rh], a.eps, a.bad);
}

// R pairs of rows [ra, ra + 2R) per wavefront, pipelined; the run's per-row
// operands and results are held one per lane, so they are read and written
// coalesced
template <int MODE, typename WT, typename IT>
__global__ void __launch_bounds__(FWD_THREADS)
k_forward_run(const int *__restrict__ row_ptr, const IT *__restrict__ col, const WT *__restrict__ val,
              const int *__restrict__ row_sino, int r0, int r1, int R, FwdArgs a) {
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t ra64 = (int64_t)r0 + ((int64_t)blockIdx.x * FWD_WAVES_PER_BLOCK + wv) * 2 * R;
    const int nr = ra64 < r1 ? (int)min((int64_t)2 * R, (int64_t)r1 - ra64) : 0;
    const int ra = nr > 0 ? (int)ra64 : r0;
    float gl = 0.0f, wl = 0.0f;
    int sl = 0;
    if (lane < nr) {
        if (MODE == 0) sl = row_sino[ra + lane];
        else { gl = a.g[ra + lane]; wl = a.w[ra + lane]; }
    }
    if (nr == 0) return;  // wave-uniform
    float outv = 0.0f;
    double term = 0.0;
    fwd_run<WT, IT>(row_ptr, col, val, a.f, ra, nr, lane, [&](int i, double s0, double s1) {
        if (lane != 2 * i && lane != 2 * i + 1) return;
        const double acc = lane == 2 * i ? s0 : s1;
        if (MODE == 0) outv = (float)acc;
        else if (MODE == 1) outv = lik_ratio(gl, wl, acc + (double)wl, a.eps);
        else term = loglik_term(gl, wl, acc + (double)wl, a.eps, a.bad);
    });
    if (lane >= nr) return;
    if (MODE == 0) a.out[sl] = outv;
    else if (MODE == 1) a.out[ra + lane] = outv;
    else a.part[ra - r0 + lane] = term;
}

// Whether a forward pass over `rows` rows runs a pair of rows per wavefront:
// by default when the rows are more than twice the wavefronts the device
// holds at once (8 per SIMD), i.e. the whole-matrix passes at the usual
// sizes, whose time is set by the bytes each wavefront streams per lifetime.
// A pass that fits runs one row per wavefront (its time is one wavefront's
// latency chain).  The persistent epoch kernel takes the same decision for
// its passes.
bool forward_pairs(const Matrix &A, int rows) { return forward_pairs_for(rows, A.pair_rows_eff()); }

// Row pairs per wavefront of a pass that runs in pairs: the tuned run length,
// by default 1 (the run kernel holds two pairs' operands in registers, which
// costs occupancy; svr_matrix_tune measures whether runs pay off).
int forward_run_length(const Matrix &A, int rows) {
    (void)rows;
    return A.run_fwd > 0 ? std::min(A.run_fwd, 31) : 1;
}

template <int MODE>
static int launch_forward_t(const Matrix &A, int r0, int r1, bool pair, int R, const FwdArgs &a, hipStream_t s,
                            int nb) {
    // one row per wavefront: XCD bin bands when the range is whole views of at
    // least XCDS bins (every subset range and the whole matrix)
    const int B = A.geom.n_bins, rows = r1 - r0;
    const bool bands = !pair && A.xcd_bands && B >= XCDS && rows % B == 0;
    const int Bb = bands ? B : 0, Vt = bands ? rows / B : 0;
    if (bands) {
        const int64_t per_xcd = ((int64_t)Vt * ((B + XCDS - 1) / XCDS) + FWD_WAVES_PER_BLOCK - 1) / FWD_WAVES_PER_BLOCK;
        nb = (int)(per_xcd * XCDS);
    }
    return with_types(A, [&](auto w, auto i) {
        using WT = decltype(w);
        using IT = decltype(i);
        if (!pair) {  // the tuned loads per lane and batch (the width never changes a row's sum)
            const IT *col = (const IT *)A.d_colt;
            const WT *val = (const WT *)A.d_val;
            if (A.sub_fwd_u == 4)
                SVR_HIP(launch_k(k_forward<MODE, false, WT, IT, 4>, nb, FWD_THREADS, s, A.d_row_ptr, col, val,
                                 A.d_row_sino, r0, r1, Bb, Vt, a));
            else if (A.sub_fwd_u == 6)
                SVR_HIP(launch_k(k_forward<MODE, false, WT, IT, 6>, nb, FWD_THREADS, s, A.d_row_ptr, col, val,
                                 A.d_row_sino, r0, r1, Bb, Vt, a));
            else
                SVR_HIP(launch_k(k_forward<MODE, false, WT, IT, FWD_U>, nb, FWD_THREADS, s, A.d_row_ptr, col, val,
                                 A.d_row_sino, r0, r1, Bb, Vt, a));
        } else if (R == 1)
            SVR_HIP(launch_k(k_forward<MODE, true, WT, IT>, nb, FWD_THREADS, s, A.d_row_ptr, (const IT *)A.d_colt,
                             (const WT *)A.d_val, A.d_row_sino, r0, r1, 0, 0, a));
        else
            SVR_HIP(launch_k(k_forward_run<MODE, WT, IT>, nb, FWD_THREADS, s, A.d_row_ptr, (const IT *)A.d_colt,
                             (const WT *)A.d_val, A.d_row_sino, r0, r1, R, a));
        return SVR_OK;
    });
}

int launch_forward(const Matrix &A, int r0, int r1, int mode, const FwdArgs &a, hipStream_t s, int *nbo) {
    const int rows = r1 - r0;
    const bool pair = rows > 0 && forward_pairs(A, rows);
    const int R = pair ? forward_run_length(A, rows) : 1;
    const int64_t waves = !pair ? (int64_t)std::max(rows, 0) : (((int64_t)rows + 1) / 2 + R - 1) / R;
    const int nb = (int)((waves + FWD_WAVES_PER_BLOCK - 1) / FWD_WAVES_PER_BLOCK);
    if (nbo) *nbo = mode == 2 ? rows : nb;
    if (nb == 0) return SVR_OK;
    if (mode == 0) return launch_forward_t<0>(A, r0, r1, pair, R, a, s, nb);
    if (mode == 1) return launch_forward_t<1>(A, r0, r1, pair, R, a, s, nb);
    return launch_forward_t<2>(A, r0, r1, pair, R, a, s, nb);
}

// x[n] = sum over subset t's transposed row (t = -1: all subsets, in t order,
// pipelined over t)
template <typename WT, typename IT>
__global__ void __launch_bounds__(BP_THREADS)
k_backproject(const int *__restrict__ ptrT, const IT *__restrict__ rowT, const WT *__restrict__ valT,
              const int *__restrict__ row_start, int Ns, int N, int t, const float *__restrict__ y_sub,
              float *__restrict__ x) {
    const int gid = blockIdx.x * BP_THREADS + threadIdx.x;
    const int n = gid / BP_G, lig = gid % BP_G;
    if (n >= N) return;  // whole groups leave together
    double acc = 0.0;
    bp_run<WT, IT>(ptrT, rowT, valT, t >= 0 ? 1 : Ns, lig, y_sub,
                   [&](int i, int64_t &q, const float *&y, float &) {
                       const int tt = t >= 0 ? t : i;
                       q = (int64_t)tt * N + n;
                       y = t >= 0 ? y_sub : y_sub + row_start[tt];
                       return true;
                   },
                   [&](int, double b, float) { acc = t >= 0 ? b : acc + b; });
    if (lig == 0) x[n] = (float)acc;
}

int launch_backproject(const Matrix &A, int t, const float *y_sub, float *x, hipStream_t s) {
    const int nb = (int)(((int64_t)A.N * BP_G + BP_THREADS - 1) / BP_THREADS);
    const float *ysub = (t >= 0) ? y_sub + A.row_start[t] : y_sub;
    return with_types(A, [&](auto w, auto i) {
        using WT = decltype(w);
        using IT = decltype(i);
        SVR_HIP(launch_k(k_backproject<WT, IT>, nb, BP_THREADS, s, A.d_ptrT, (const IT *)A.d_rowT,
                         (const WT *)A.d_valT, A.d_row_start, A.Ns, A.N, t, ysub, x));
        return SVR_OK;
    });
}

// penalty value partials: one FP64 partial per block of 256 pixels
__global__ void __launch_bounds__(256) k_penalty_value(const float *f, int N, PenaltyArgs p, double *part) {
    __shared__ double red[256];
    const int n = blockIdx.x * 256 + threadIdx.x;
    red[threadIdx.x] = (n < N) ? penalty_share_at(f, n, p) : 0.0;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

int launch_penalty_value(const Matrix &A, const float *f, int potential, double delta, double *part,
                         int *nbo, hipStream_t s) {
    PenaltyArgs p{potential, delta, 0.0, A.geom.nx, A.geom.ny};
    const int nb = (A.N + 255) / 256;
    *nbo = nb;
    k_penalty_value<<<nb, 256, 0, s>>>(f, A.N, p, part);
    SVR_HIP(hipGetLastError());
    return SVR_OK;
}

}  // namespace svr
