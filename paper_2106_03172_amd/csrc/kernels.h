// Device building blocks shared by the projector and update kernels.  Every
// reduction here has a fixed order, so a quantity computed by two different
// kernels (an anchor table entry and the same quantity in a later iteration)
// is bitwise identical.
//
// The sparse loops are written load-phase-first: each lane issues all index
// and weight loads of a batch, then all gathers, then the FP64 products, so a
// wavefront keeps FWD_U (or BP_U) independent loads in flight per lane
// instead of walking a dependent index -> gather chain entry by entry.  The
// entries a lane visits, and their order, are the same as a plain strided
// loop.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "common.h"

namespace svr {

#ifndef SVR_FWD_U
#define SVR_FWD_U 8
#endif
#ifndef SVR_BP_G
#define SVR_BP_G 4
#endif
#ifndef SVR_BP_U
#define SVR_BP_U 8
#endif
constexpr int FWD_THREADS = 256;               // forward: 4 wavefronts per block
constexpr int FWD_ROWS_PER_BLOCK = FWD_THREADS / 64;
constexpr int FWD_U = SVR_FWD_U;               // loads in flight per lane (64*8 = 512 nnz per batch)
constexpr int BP_G = SVR_BP_G;                 // back-projection lanes per pixel
constexpr int BP_U = SVR_BP_U;                 // loads in flight per lane (4*8 = 32 nnz per batch)
constexpr int BP_THREADS = 256;

// ---- launches, optionally timed by events attached to the dispatch itself ----
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
LaunchEvents &pending_timing();  // per host thread (util.hip)

template <typename... KArgs, typename... Args>
inline hipError_t launch_k(void (*kernel)(KArgs...), dim3 grid, dim3 block, hipStream_t s, Args... args) {
    LaunchEvents &t = pending_timing();
    if (t.start) {
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, t.start, t.stop, 0, static_cast<KArgs>(args)...);
        t.start = t.stop = nullptr;
    } else {
        kernel<<<grid, block, 0, s>>>(static_cast<KArgs>(args)...);
    }
    return hipGetLastError();
}

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v = v + __shfl_xor(v, o, 64);
    return v;
}

// (A f)_r: the lanes of a wavefront stride over row r's non-zeros, FP64 products
template <typename WT, typename IT>
__device__ inline double row_dot(const int *__restrict__ row_ptr, const IT *__restrict__ col,
                                 const WT *__restrict__ val, const float *__restrict__ f, int r, int lane) {
    const int beg = row_ptr[r], end = row_ptr[r + 1];
    double acc = 0.0;
    for (int base = beg + lane; base < end; base += 64 * FWD_U) {
        int c[FWD_U];
        float v[FWD_U], x[FWD_U];
#pragma unroll
        for (int u = 0; u < FWD_U; ++u) {
            const int i = base + 64 * u;
            c[u] = i < end ? (int)col[i] : -1;
            v[u] = i < end ? load_w(val[i]) : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < FWD_U; ++u) x[u] = c[u] >= 0 ? f[c[u]] : 0.0f;
#pragma unroll
        for (int u = 0; u < FWD_U; ++u)
            if (c[u] >= 0) acc = acc + (double)v[u] * (double)x[u];
    }
    return acc;
}

// EM ratio g / ybar with the zero-denominator rule (0 if g == 0 or ybar <= 0)
__device__ inline float em_ratio(float g, double yb) {
    return (g > 0.0f && yb > 0.0) ? (float)((double)g / yb) : 0.0f;
}

// Forward row r with the EM ratio written to ratio[r]; every lane of the
// wavefront calls it with the same r.
template <typename WT, typename IT>
__device__ inline void fwd_ratio_row(const int *__restrict__ row_ptr, const IT *__restrict__ col,
                                     const WT *__restrict__ val, const float *__restrict__ f,
                                     const float *__restrict__ g, const float *__restrict__ w,
                                     float *__restrict__ ratio, int r, int lane) {
    const float gv = g[r], wv = w[r];
    double acc = row_dot(row_ptr, col, val, f, r, lane);
    acc = wave_sum(acc);
    if (lane == 0) ratio[r] = em_ratio(gv, acc + (double)wv);
}

// sum over transposed row q of val * y[row], BP_G lanes per row; every lane
// of the group returns the same value
template <typename WT, typename IT>
__device__ inline double bp_group(const int *__restrict__ ptrT, const IT *__restrict__ rowT,
                                  const WT *__restrict__ valT, int64_t q, const float *__restrict__ y,
                                  int lig) {
    const int beg = ptrT[q], end = ptrT[q + 1];
    double acc = 0.0;
    for (int base = beg + lig; base < end; base += BP_G * BP_U) {
        int rr[BP_U];
        float v[BP_U], x[BP_U];
#pragma unroll
        for (int u = 0; u < BP_U; ++u) {
            const int i = base + BP_G * u;
            rr[u] = i < end ? (int)rowT[i] : -1;
            v[u] = i < end ? load_w(valT[i]) : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < BP_U; ++u) x[u] = rr[u] >= 0 ? y[rr[u]] : 0.0f;
#pragma unroll
        for (int u = 0; u < BP_U; ++u)
            if (rr[u] >= 0) acc = acc + (double)v[u] * (double)x[u];
    }
    for (int o = BP_G / 2; o > 0; o >>= 1) acc = acc + __shfl_xor(acc, o, 64);
    return acc;
}

}  // namespace svr
