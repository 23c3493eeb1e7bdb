// Projectors: forward rows of A (with the fused EM ratio or log-likelihood)
// and the gather-only transposed back-projection.
//
// Forward: one 64-lane wavefront per row of A, lanes striding over the row's
// non-zeros (coalesced reads of the index and weight streams, image gathers
// from L2), FP64 products and a fixed butterfly reduction, so a row always
// sums in the same order whichever call computes it.
//
// Back-projection: BP_G lanes per pixel over that pixel's transposed row of
// subset t, FP64 products, fixed butterfly reduction.
#include <cmath>

#include "common.h"
#include "kernels.h"
#include "penalty.h"

namespace svr {

template <int MODE, typename WT, typename IT>
__global__ void __launch_bounds__(FWD_THREADS)
k_forward(const int *__restrict__ row_ptr, const IT *__restrict__ col, const WT *__restrict__ val,
          const int *__restrict__ row_sino, int r0, int r1, FwdArgs a) {
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int r = r0 + blockIdx.x * FWD_ROWS_PER_BLOCK + wv;
    if (MODE == 1) {  // wave-uniform: the wave either has a row or not
        if (r < r1) fwd_ratio_row(row_ptr, col, val, a.f, a.g, a.w, a.out, r, lane);
        return;
    }
    double acc = 0.0;
    if (r < r1) acc = row_dot(row_ptr, col, val, a.f, r, lane);
    acc = wave_sum(acc);
    if (MODE == 0) {
        if (lane == 0 && r < r1) a.out[row_sino[r]] = (float)acc;
    } else {
        __shared__ double part[FWD_ROWS_PER_BLOCK];
        if (lane == 0) {
            double term = 0.0;
            if (r < r1) {
                const double yb = acc + (double)a.w[r];
                const float gv = a.g[r];
                if (gv > 0.0f) {
                    if (yb > 0.0) term = (double)gv * log(yb) - yb;
                    else { atomicOr(a.bad, 1); term = 0.0; }
                } else {
                    term = -yb;
                }
            }
            part[wv] = term;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int i = 0; i < FWD_ROWS_PER_BLOCK; ++i) s = s + part[i];
            a.part[blockIdx.x] = s;
        }
    }
}

template <int MODE>
static int launch_forward_t(const Matrix &A, int r0, int r1, const FwdArgs &a, hipStream_t s, int nb) {
    return with_types(A, [&](auto w, auto i) {
        using WT = decltype(w);
        using IT = decltype(i);
        SVR_HIP(launch_k(k_forward<MODE, WT, IT>, nb, FWD_THREADS, s, A.d_row_ptr, (const IT *)A.d_col,
                         (const WT *)A.d_val, A.d_row_sino, r0, r1, a));
        return SVR_OK;
    });
}

int launch_forward(const Matrix &A, int r0, int r1, int mode, const FwdArgs &a, hipStream_t s, int *nbo) {
    const int rows = r1 - r0;
    const int nb = rows > 0 ? (rows + FWD_ROWS_PER_BLOCK - 1) / FWD_ROWS_PER_BLOCK : 0;
    if (nbo) *nbo = nb;
    if (nb == 0) return SVR_OK;
    if (mode == 0) return launch_forward_t<0>(A, r0, r1, a, s, nb);
    if (mode == 1) return launch_forward_t<1>(A, r0, r1, a, s, nb);
    return launch_forward_t<2>(A, r0, r1, a, s, nb);
}

// x[n] = sum over subset t's transposed row (t = -1: all subsets, in t order)
template <typename WT, typename IT>
__global__ void __launch_bounds__(BP_THREADS)
k_backproject(const int *__restrict__ ptrT, const IT *__restrict__ rowT, const WT *__restrict__ valT,
              const int *__restrict__ row_start, int Ns, int N, int t, const float *__restrict__ y_sub,
              float *__restrict__ x) {
    const int gid = blockIdx.x * BP_THREADS + threadIdx.x;
    const int n = gid / BP_G, lig = gid % BP_G;
    if (n >= N) return;
    double acc = 0.0;
    if (t >= 0) {
        acc = bp_group(ptrT, rowT, valT, (int64_t)t * N + n, y_sub, lig);
    } else {
        for (int tt = 0; tt < Ns; ++tt)
            acc = acc + bp_group(ptrT, rowT, valT, (int64_t)tt * N + n, y_sub + row_start[tt], lig);
    }
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
