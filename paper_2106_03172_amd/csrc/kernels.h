// Device building blocks shared by the projector and update kernels.  Every
// reduction here has a fixed order, so a quantity computed by two kernels
// through the same function (a back-projected table entry at an anchor and
// the same back-projection in a later iteration; a forward row in the
// per-phase and in the persistent kernels) is bitwise identical.
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
#ifndef SVR_FWD_PAIR_U
#define SVR_FWD_PAIR_U 12
#endif
#ifndef SVR_BP_G
#define SVR_BP_G 4
#endif
#ifndef SVR_BP_U
#define SVR_BP_U 5
#endif
constexpr int FWD_THREADS = 256;               // forward: 4 wavefronts per block
constexpr int FWD_WAVES_PER_BLOCK = FWD_THREADS / 64;
constexpr int FWD_U = SVR_FWD_U;               // loads in flight per lane, one row per wavefront (64*8 = 512
                                               // entries per batch: the longest row of the 256x256 matrix)
constexpr int FWD_PAIR_U = SVR_FWD_PAIR_U;     // the same for a pair of rows (32*12 = 384 entries of each)
constexpr int BP_G = SVR_BP_G;                 // back-projection lanes per pixel
constexpr int BP_U = SVR_BP_U;                 // loads in flight per lane (4*5 = 20 nnz per batch: one
                                               // batch covers a whole transposed subset row of a 2 mm
                                               // 256x256 image, 252 views, 21 subsets, in >99% of rows;
                                               // 5 beat 4, 6, 7 and 8 in measured anchor-table time)
constexpr int BP_THREADS = 256;
#ifndef SVR_FWD_RUN_U
#define SVR_FWD_RUN_U 8
#endif
#ifndef SVR_BP_RUN_U
#define SVR_BP_RUN_U 5
#endif
constexpr int FWD_RUN_U = SVR_FWD_RUN_U;       // loads in flight per lane and batch in the row runs
constexpr int BP_RUN_U = SVR_BP_RUN_U;         // 4*5 = 20, as BP_U (46.5 -> 39 us per whole back-projection)

// ---- launches, optionally timed by events attached to the dispatch itself ----
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
    int span = 1;  // launches the armed pair covers: start on the first, stop on the last
};
LaunchEvents &pending_timing();  // per host thread (util.hip)

template <typename... KArgs, typename... Args>
inline hipError_t launch_k(void (*kernel)(KArgs...), dim3 grid, dim3 block, hipStream_t s, Args... args) {
    LaunchEvents &t = pending_timing();
    if (t.start || t.stop) {
        hipEvent_t stop = t.span <= 1 ? t.stop : nullptr;
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, t.start, stop, 0, static_cast<KArgs>(args)...);
        t.start = nullptr;
        if (t.span <= 1) {
            t.stop = nullptr;
            t.span = 1;
        } else {
            --t.span;
        }
    } else {
        kernel<<<grid, block, 0, s>>>(static_cast<KArgs>(args)...);
    }
    return hipGetLastError();
}

// ---- XCD-contiguous work chunks ----------------------------------------------------
// Workgroups are dispatched to the XCDs round-robin by index.  A pass over
// `chunks` consecutive chunks of work launched as xcd_grid(chunks, per) blocks
// gives block b the chunk xcd_chunk(b, per): XCD b mod XCDS takes the
// contiguous chunks [x per, (x + 1) per), so the cache lines two neighbouring
// chunks share, and the image rows a pixel's stencil reads, stay in one L2.
// Past the last chunk: >= chunks (the block returns).  Which block takes a
// chunk changes nothing in its arithmetic.
__device__ inline int xcd_chunk(int b, int per) { return (b % XCDS) * per + b / XCDS; }
inline int xcd_grid(int64_t chunks, int &per) {
    per = (int)((chunks + XCDS - 1) / XCDS);
    return per * XCDS;
}

// ---- cross-lane sums ------------------------------------------------------------
// FP64 value of another lane through a DPP move of both halves (CTRL: the
// GFX9 DPP control; every source lane used here lies in the same 16-lane row
// and is active whenever the reading lane is).
template <int CTRL>
__device__ inline double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
constexpr int DPP_XOR1 = 0xB1;         // quad_perm [1,0,3,2]: lane ^ 1
constexpr int DPP_XOR2 = 0x4E;         // quad_perm [2,3,0,1]: lane ^ 2
constexpr int DPP_HALF_MIRROR = 0x141;  // lane i <-> 7 - i within each 8
constexpr int DPP_MIRROR = 0x140;       // lane i <-> 15 - i within each 16

__device__ inline double readlane_f64(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sums over the two 32-lane halves of a wavefront, the same values in every
// lane, in a fixed order: lane pairs, quads, 8s and 16s by DPP moves (after
// each step every lane of the group holds the group's sum: a + b and b + a
// are the same number), then the 16-lane rows as s0 = r0 + r1 (lanes 0-31)
// and s1 = r2 + r3 (lanes 32-63).  Every lane of the wavefront must call it
// (the rows are read with readlane).  DPP moves stay in the vector ALU; a
// shuffle would go through the LDS crossbar, one round trip per 32-bit half
// and step.
__device__ inline void half_sums(double v, double &s0, double &s1) {
    v = v + dpp_f64<DPP_XOR1>(v);
    v = v + dpp_f64<DPP_XOR2>(v);
    v = v + dpp_f64<DPP_HALF_MIRROR>(v);
    v = v + dpp_f64<DPP_MIRROR>(v);
    s0 = readlane_f64(v, 0) + readlane_f64(v, 16);
    s1 = readlane_f64(v, 32) + readlane_f64(v, 48);
}

// Sum over the 64 lanes of a wavefront, (r0 + r1) + (r2 + r3) as above.
__device__ inline double wave_sum(double v) {
    double s0, s1;
    half_sums(v, s0, s1);
    return s0 + s1;
}

// ---- range-checked buffer loads ----------------------------------------------
// A raw buffer resource over `bytes` bytes from p: a buffer load whose byte
// offset is at or past `bytes` returns 0 and makes no memory request (the
// hardware's range check of raw buffers, stride 0).  A wavefront that owns a
// row builds one over the rest of that row, so every slot of a batch is issued
// unconditionally (no per-lane branch) while the slots past the row's end cost
// no cache lines.  Word 3 selects a 32-bit data format, which untyped loads
// need to be non-zero; the offset and swizzle fields stay 0.
constexpr int BUF_RSRC_WORD3 = 0x00020000;
__device__ inline __amdgpu_buffer_rsrc_t range_rsrc(const void *p, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, BUF_RSRC_WORD3);
}
template <typename T>
__device__ inline T buf_load(__amdgpu_buffer_rsrc_t r, int off);
template <>
__device__ inline uint16_t buf_load<uint16_t>(__amdgpu_buffer_rsrc_t r, int off) {
    return (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
}
template <>
__device__ inline int buf_load<int>(__amdgpu_buffer_rsrc_t r, int off) {
    return (int)__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}
template <>
__device__ inline float buf_load<float>(__amdgpu_buffer_rsrc_t r, int off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ inline _Float16 buf_load<_Float16>(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(_Float16, (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
}
template <>
__device__ inline bf16_t buf_load<bf16_t>(__amdgpu_buffer_rsrc_t r, int off) {
    return bf16_t{(uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0)};
}

// One batch of a sparse row held in registers: lane j of an L-lane team
// holds entries base + j + L*u (u < U) of the row ending at `end`, index -1
// past the end.  Every sparse sum in the library walks its rows batch by
// batch through this struct, so a row's products are always added in the
// same order, whichever kernel (and whichever pipelining) computes it.
template <int L, int U, typename WT, typename IT>
struct RowBatch {
    int c[U];
    float v[U];
    // Every load is unconditional (the arrays carry NNZ_PAD zero entries
    // after the last row, so a batch may read past a row's end; the image or
    // ratio gather of an invalid entry reads element 0): a load behind a
    // per-lane branch makes the compiler wait for it before the branches
    // join, which would serialise the batch.
    __device__ inline void load(const IT *__restrict__ idx, const WT *__restrict__ val, int base, int end) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + L * u;
            const int ci = (int)idx[i];
            const float vi = load_w(val[i]);
            c[u] = i < end ? ci : -1;
            v[u] = vi;
        }
    }
    // The batch of a row owned by the whole wavefront (L = 64): entries
    // bb + lane + 64 u of the row ending at `end` (bb, end wavefront-uniform),
    // the entries and lanes of load(idx, val, bb + lane, end), read through
    // range-checked resources that end at the row's end.
    __device__ inline void load_wave(const IT *__restrict__ idx, const WT *__restrict__ val, int bb, int end,
                                     int lane) {
        const int n = end - bb;
        const __amdgpu_buffer_rsrc_t ri = range_rsrc(idx + bb, n * (int)sizeof(IT));
        const __amdgpu_buffer_rsrc_t rv = range_rsrc(val + bb, n * (int)sizeof(WT));
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int o = lane + L * u;
            const int ci = (int)buf_load<IT>(ri, o * (int)sizeof(IT));
            const float vi = load_w(buf_load<WT>(rv, o * (int)sizeof(WT)));
            c[u] = o < n ? ci : -1;
            v[u] = vi;
        }
    }
    // One batch of a pair of consecutive rows owned by a wavefront (L = 32):
    // the row of half h = lane >> 5 spans [b0, e0) (h = 0) or [e0, e1)
    // (h = 1), and lane hl = lane & 31 holds its entries beg_h + k + hl + 32 u.
    // Both halves read through one range-checked resource from the first
    // row's batch start b0 + k to the second row's end, so slots past a row's
    // end fetch the other row's entries (masked) or nothing.  b0, e0, e1 and
    // k are wavefront-uniform.
    __device__ inline void load_pair(const IT *__restrict__ idx, const WT *__restrict__ val, int b0, int e0, int e1,
                                     int k, int lane) {
        static_assert(L == 32, "a pair batch has 32 lanes per row");
        const int h = lane >> 5, hl = lane & 31;
        const int wb = b0 + k, n = max(e1 - wb, 0);
        const __amdgpu_buffer_rsrc_t ri = range_rsrc(idx + wb, n * (int)sizeof(IT));
        const __amdgpu_buffer_rsrc_t rv = range_rsrc(val + wb, n * (int)sizeof(WT));
        const int beg = h ? e0 : b0, end = h ? e1 : e0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = beg + k + hl + L * u;
            const int o = i - wb;
            const int ci = (int)buf_load<IT>(ri, o * (int)sizeof(IT));
            const float vi = load_w(buf_load<WT>(rv, o * (int)sizeof(WT)));
            c[u] = i < end ? ci : -1;
            v[u] = vi;
        }
    }
    __device__ inline void gather(const float *__restrict__ x, float (&xv)[U]) const {
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = x[c[u] >= 0 ? c[u] : 0];
    }
    // acc + v*x with one FP64 fused multiply-add: the product of two FP32
    // values is exact in FP64, so this rounds exactly like a multiply
    // followed by an add
    __device__ inline double fma(const float (&xv)[U], double acc) const {
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (c[u] >= 0) acc = __builtin_fma((double)v[u], (double)xv[u], acc);
        return acc;
    }
};

// the batches of a row after its first, starting at lane offset `first`
template <int L, int U, typename WT, typename IT>
__device__ inline double row_rest(const IT *__restrict__ idx, const WT *__restrict__ val, const float *__restrict__ x,
                                  int first, int end, double acc) {
    for (int base = first + L * U; base < end; base += L * U) {
        RowBatch<L, U, WT, IT> b;
        float xv[U];
        b.load(idx, val, base, end);
        b.gather(x, xv);
        acc = b.fma(xv, acc);
    }
    return acc;
}

// ---- forward rows ----------------------------------------------------------------
// (A f)_r: the lanes of a wavefront stride over row r's non-zeros in batches
// of 64 * U (U = FWD_U unless tuned), FP64 products; lane j adds entries
// beg + j, beg + j + 64, ... in that order whatever U.  The per-subset passes,
// whose rows fit in the wavefronts the device holds at once, run one row per
// wavefront: their time is one wavefront's latency chain, which a pair per
// wavefront lengthens.
template <int U = FWD_U, typename WT, typename IT>
__device__ inline double row_dot(const int *__restrict__ row_ptr, const IT *__restrict__ col,
                                 const WT *__restrict__ val, const float *__restrict__ f, int r, int lane) {
    r = __builtin_amdgcn_readfirstlane(r);  // one row per wavefront: scalar row bounds
    const int beg = row_ptr[r], end = row_ptr[r + 1];
    double acc = 0.0;
    for (int bb = beg; bb < end; bb += 64 * U) {
        RowBatch<64, U, WT, IT> b;
        float xv[U];
        b.load_wave(col, val, bb, end, lane);
        b.gather(f, xv);
        acc = b.fma(xv, acc);
    }
    return acc;
}

// ---- forward rows in pairs ------------------------------------------------------
// A wavefront owns a pair of consecutive rows r, r + 1 of A: the 32 lanes of
// half h = lane >> 5 take row r + h, lane hl = lane & 31 adding the entries
// beg + hl, beg + hl + 32, ... of its row in that order (FP64 fused
// multiply-adds), and half_sums adds each half's lanes.  A whole-matrix pass
// is bounded by the index/weight bytes a wavefront streams per lifetime (row
// pointers -> index/weight -> gathers -> sum); a pair per wavefront doubles
// them.

// lane partial of the pair with bounds b0 <= e0 <= e1 (e1 == e0: no second
// row), all wavefront-uniform
template <typename WT, typename IT>
__device__ inline double pair_dot(const IT *__restrict__ col, const WT *__restrict__ val,
                                  const float *__restrict__ f, int b0, int e0, int e1, int lane) {
    const int len = max(e0 - b0, e1 - e0);
    double acc = 0.0;
    for (int k = 0; k < len; k += 32 * FWD_PAIR_U) {
        RowBatch<32, FWD_PAIR_U, WT, IT> b;
        float xv[FWD_PAIR_U];
        b.load_pair(col, val, b0, e0, e1, k, lane);
        b.gather(f, xv);
        acc = b.fma(xv, acc);
    }
    return acc;
}

// sum over t < Ns of x[t * stride + i], FP64, added in t order.  The loads
// are issued 16 at a time (indices clamped in bounds, the extra values not
// added): a load per iteration would wait for each one before the next add.
template <class Mid>
__device__ inline double subset_sum_mid(const float *__restrict__ x, int Ns, int64_t stride, int64_t i, Mid mid) {
    constexpr int B = 32;  // one round trip for up to 32 subsets
    double sum = 0.0;
    for (int t0 = 0; t0 < Ns; t0 += B) {
        float v[B];
#pragma unroll
        for (int k = 0; k < B; ++k) v[k] = x[(int64_t)min(t0 + k, Ns - 1) * stride + i];
        if (t0 == 0) mid();  // while the first batch is in flight
#pragma unroll
        for (int k = 0; k < B; ++k)
            if (t0 + k < Ns) sum = sum + (double)v[k];
    }
    return sum;
}

__device__ inline double subset_sum(const float *__restrict__ x, int Ns, int64_t stride, int64_t i) {
    return subset_sum_mid(x, Ns, stride, i, [] {});
}

// EM ratio g / ybar with the zero-denominator rule (0 if g == 0 or ybar <= 0)
__device__ inline float em_ratio(float g, double yb) {
    return (g > 0.0f && yb > 0.0) ? (float)((double)g / yb) : 0.0f;
}

// The ratio whose back-projection minus A^T 1 is the likelihood gradient:
// the EM ratio, or with eps > 0 (the modified likelihood of Sec. 2.3,
// eq. modified_LL) for rows with w = 0 and ybar <= eps the derivative of the
// second-order expansion about eps plus one, g (2 eps - ybar) / eps^2.
__device__ inline float lik_ratio(float g, float w, double yb, double eps) {
    if (eps > 0.0 && w == 0.0f && yb <= eps)
        return g > 0.0f ? (float)(((double)g * (2.0 * eps - yb)) / (eps * eps)) : 0.0f;
    return em_ratio(g, yb);
}

// Forward row r with the ratio written to ratio[r]; every lane of the
// wavefront calls it with the same r.
template <int U = FWD_U, typename WT, typename IT>
__device__ inline void fwd_ratio_row(const int *__restrict__ row_ptr, const IT *__restrict__ col,
                                     const WT *__restrict__ val, const float *__restrict__ f,
                                     const float *__restrict__ g, const float *__restrict__ w,
                                     float *__restrict__ ratio, int r, int lane, double eps) {
    const float gv = g[r], wv = w[r];
    double acc = row_dot<U>(row_ptr, col, val, f, r, lane);
    acc = wave_sum(acc);
    if (lane == 0) ratio[r] = lik_ratio(gv, wv, acc + (double)wv, eps);
}

// Forward of rows r and r + 1 (the second only if r + 1 < r1) with each
// row's ratio written to ratio[row]; every lane of the wavefront calls it
// with the same r < r1.
template <typename WT, typename IT>
__device__ inline void fwd_ratio_pair(const int *__restrict__ row_ptr, const IT *__restrict__ col,
                                      const WT *__restrict__ val, const float *__restrict__ f,
                                      const float *__restrict__ g, const float *__restrict__ w,
                                      float *__restrict__ ratio, int r, int r1, int lane, double eps) {
    r = __builtin_amdgcn_readfirstlane(r);  // scalar row bounds
    const int h = lane >> 5, rh = r + h;
    const int rl = min(rh, r1 - 1);  // in bounds; a missing second row writes nothing
    const float gv = g[rl], wv = w[rl];
    const int b0 = row_ptr[r], e0 = row_ptr[r + 1], e1 = row_ptr[min(r + 2, r1)];
    double s0, s1;
    half_sums(pair_dot(col, val, f, b0, e0, e1, lane), s0, s1);
    if ((lane & 31) == 0 && rh < r1) ratio[rh] = lik_ratio(gv, wv, (h ? s1 : s0) + (double)wv, eps);
}

// Sum over the BP_G lanes of a back-projection group (xor butterfly, every
// lane of the group gets the same value); groups are aligned to BP_G lanes.
__device__ inline double group_sum(double acc) {
    static_assert(BP_G == 1 || BP_G == 2 || BP_G == 4 || BP_G == 8 || BP_G == 16, "BP_G: 1, 2, 4, 8 or 16");
    if constexpr (BP_G >= 16) acc = acc + dpp_f64<DPP_MIRROR>(acc);
    if constexpr (BP_G >= 8) acc = acc + dpp_f64<DPP_HALF_MIRROR>(acc);
    if constexpr (BP_G >= 4) acc = acc + dpp_f64<DPP_XOR2>(acc);
    if constexpr (BP_G >= 2) acc = acc + dpp_f64<DPP_XOR1>(acc);
    return acc;
}

// sum over transposed row q of val * y[row], BP_G lanes per row; every lane
// of the group returns the same value
template <typename WT, typename IT>
__device__ inline double bp_range(const IT *__restrict__ rowT, const WT *__restrict__ valT, int beg, int end,
                                  const float *__restrict__ y, int lig) {
    double acc = 0.0;
    for (int base = beg + lig; base < end; base += BP_G * BP_U) {
        RowBatch<BP_G, BP_U, WT, IT> b;
        float xv[BP_U];
        b.load(rowT, valT, base, end);
        b.gather(y, xv);
        acc = b.fma(xv, acc);
    }
    return group_sum(acc);
}

// The same sum with `mid()` run once per lane while the lane's first
// index/weight batch is in flight (after the loop for a lane with no entries):
// work that does not depend on the sum, such as the penalty's stencil sums,
// then takes none of the gather's latency.  U entries per lane and batch
// (BP_U unless tuned); lane lig adds entries beg + lig, beg + lig + BP_G, ...
// in that order whatever U.
template <int U = BP_U, typename WT, typename IT, class Mid>
__device__ inline double bp_range_mid(const IT *__restrict__ rowT, const WT *__restrict__ valT, int beg, int end,
                                      const float *__restrict__ y, int lig, Mid mid) {
    double acc = 0.0;
    bool done = false;
    for (int base = beg + lig; base < end; base += BP_G * U) {
        RowBatch<BP_G, U, WT, IT> b;
        float xv[U];
        b.load(rowT, valT, base, end);
        if (!done) {
            mid();
            done = true;
        }
        b.gather(y, xv);
        acc = b.fma(xv, acc);
    }
    if (!done) mid();
    return group_sum(acc);
}

template <typename WT, typename IT>
__device__ inline double bp_group(const int *__restrict__ ptrT, const IT *__restrict__ rowT,
                                  const WT *__restrict__ valT, int64_t q, const float *__restrict__ y,
                                  int lig) {
    return bp_range(rowT, valT, ptrT[q], ptrT[q + 1], y, lig);
}

// ---- pipelined row runs -------------------------------------------------------
// A wavefront that owns a run of rows [ra, ra + nr) of A (nr <= 62) walks it
// in pairs (ra + 2i, ra + 2i + 1) with the first index/weight batch of pair
// i + 1 in flight while it gathers and sums pair i (the run's row pointers
// are loaded up front, one per lane), so each pair costs about one memory
// latency instead of three.  The entries each lane adds, and their order, are
// pair_dot's.  `fin(i, s0, s1)` gets the sums of pair i's two rows (s1 = 0
// for a missing second row).
template <typename WT, typename IT, class Fin>
__device__ inline void fwd_run(const int *__restrict__ row_ptr, const IT *__restrict__ col, const WT *__restrict__ val,
                               const float *__restrict__ f, int ra, int nr, int lane, Fin fin) {
    const int rp = row_ptr[ra + min(lane, nr)];  // lanes past nr repeat the run's end
    const int np = (nr + 1) / 2;
    auto bounds = [&](int i, int &b0, int &e0, int &e1) {
        b0 = __builtin_amdgcn_readlane(rp, 2 * i);
        e0 = __builtin_amdgcn_readlane(rp, min(2 * i + 1, nr));
        e1 = __builtin_amdgcn_readlane(rp, min(2 * i + 2, nr));
    };
    int b0, e0, e1;
    bounds(0, b0, e0, e1);
    RowBatch<32, FWD_RUN_U, WT, IT> cur;
    cur.load_pair(col, val, b0, e0, e1, 0, lane);
    for (int i = 0; i < np; ++i) {
        float xv[FWD_RUN_U];
        cur.gather(f, xv);
        int nb0 = 0, ne0 = 0, ne1 = 0;
        RowBatch<32, FWD_RUN_U, WT, IT> nxt;
        if (i + 1 < np) {
            bounds(i + 1, nb0, ne0, ne1);
            nxt.load_pair(col, val, nb0, ne0, ne1, 0, lane);
        }
        double acc = cur.fma(xv, 0.0);
        const int len = max(e0 - b0, e1 - e0);
        for (int k = 32 * FWD_RUN_U; k < len; k += 32 * FWD_RUN_U) {  // as pair_dot
            RowBatch<32, FWD_RUN_U, WT, IT> b;
            b.load_pair(col, val, b0, e0, e1, k, lane);
            b.gather(f, xv);
            acc = b.fma(xv, acc);
        }
        double s0, s1;
        half_sums(acc, s0, s1);
        fin(i, s0, s1);
        b0 = nb0;
        e0 = ne0;
        e1 = ne1;
        cur = nxt;
    }
}

// A BP_G-lane group that owns the transposed rows q(0), q(1), ..., q(n-1)
// walks them three deep: row pointers (and one per-row operand) of step
// i+2, the index/weight batch of step i+1 and the gathers of step i are in
// flight together.  `seq(i, q, y, aux)` names step i's row, the vector it
// gathers from and loads the per-row operand `aux` (false: no row, the sum
// is 0, and the gathers read ydef[0]); `fin(i, b, aux)` gets the
// group-reduced sum.  Every lane of the
// group takes the same steps.
template <typename WT, typename IT, class Seq, class Fin>
__device__ inline void bp_run(const int *__restrict__ ptrT, const IT *__restrict__ rowT, const WT *__restrict__ valT,
                              int n, int lig, const float *ydef, Seq seq, Fin fin) {
    int64_t q;
    const float *y0 = ydef, *y1 = ydef;
    int b0 = 0, e0 = 0, b1 = 0, e1 = 0;
    float a0 = 0.0f, a1 = 0.0f;
    if (n > 0 && seq(0, q, y0, a0)) { b0 = ptrT[q]; e0 = ptrT[q + 1]; }
    if (n > 1 && seq(1, q, y1, a1)) { b1 = ptrT[q]; e1 = ptrT[q + 1]; }
    RowBatch<BP_G, BP_RUN_U, WT, IT> cur;
    cur.load(rowT, valT, b0 + lig, e0);
    for (int i = 0; i < n; ++i) {
        float xv[BP_RUN_U];
        cur.gather(y0, xv);
        RowBatch<BP_G, BP_RUN_U, WT, IT> nxt;
        nxt.load(rowT, valT, b1 + lig, e1);
        const float *y2 = ydef;
        int b2 = 0, e2 = 0;
        float a2 = 0.0f;
        if (i + 2 < n && seq(i + 2, q, y2, a2)) { b2 = ptrT[q]; e2 = ptrT[q + 1]; }
        double acc = cur.fma(xv, 0.0);
        acc = row_rest<BP_G, BP_RUN_U, WT, IT>(rowT, valT, y0, b0 + lig, e0, acc);
        fin(i, group_sum(acc), a0);
        b0 = b1; e0 = e1; y0 = y1; a0 = a1;
        b1 = b2; e1 = e2; y1 = y2; a1 = a2;
        cur = nxt;
    }
}

}  // namespace svr
