// Device building blocks shared by the projector and update kernels.  Every
// reduction here has a fixed order, so a quantity computed by two different
// kernels (an anchor table entry and the same quantity in a later iteration)
// is bitwise identical.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace svr {

constexpr int FWD_THREADS = 256;               // forward: 4 wavefronts per block
constexpr int FWD_ROWS_PER_BLOCK = FWD_THREADS / 64;
constexpr int BP_G = 4;                        // back-projection lanes per pixel
constexpr int BP_THREADS = 256;

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v = v + __shfl_xor(v, o, 64);
    return v;
}

// (A f)_r: lanes stride over row r's non-zeros, FP64 products
template <typename WT>
__device__ inline double row_dot(const int *__restrict__ row_ptr, const int *__restrict__ col,
                                 const WT *__restrict__ val, const float *__restrict__ f, int r, int lane) {
    const int beg = row_ptr[r], end = row_ptr[r + 1];
    double acc = 0.0;
    for (int i = beg + lane; i < end; i += 64) acc = acc + (double)load_w(val[i]) * (double)f[col[i]];
    return acc;
}

// EM ratio g / ybar with the zero-denominator rule (0 if g == 0 or ybar <= 0)
__device__ inline float em_ratio(float g, double yb) {
    return (g > 0.0f && yb > 0.0) ? (float)((double)g / yb) : 0.0f;
}

// sum over transposed row q of val * y[row], BP_G lanes per row; every lane
// of the group returns the same value
template <typename WT>
__device__ inline double bp_group(const int *__restrict__ ptrT, const int *__restrict__ rowT,
                                  const WT *__restrict__ valT, int64_t q, const float *__restrict__ y,
                                  int lig) {
    const int beg = ptrT[q], end = ptrT[q + 1];
    double acc = 0.0;
    for (int i = beg + lig; i < end; i += BP_G) acc = acc + (double)load_w(valT[i]) * (double)y[rowT[i]];
    for (int o = BP_G / 2; o > 0; o >>= 1) acc = acc + __shfl_xor(acc, o, 64);
    return acc;
}

}  // namespace svr
