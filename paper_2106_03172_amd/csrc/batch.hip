// Batched subset iterations (one launch per phase for several requests).
// A block finds its request by the items' first blocks (uniform across the
// block), then runs the single-request code for its rows or pixels.
#include "batch.h"
#include "kernels.h"
#include "phases.h"

namespace svr {

template <class Batch>
__device__ inline int item_of(const Batch &b) {
    int i = 0;
#pragma unroll
    for (int j = 1; j < BATCH_MAX; ++j)
        if (j < b.n && (int)blockIdx.x >= b.it[j].blk0) i = j;
    return i;
}

// forward + ratio of each item's subset rows (one row, or a pair of rows, per
// wavefront, as the item's own pass would run them)
template <typename WT, typename IT>
__global__ void __launch_bounds__(FWD_THREADS) k_forward_batch(FwdBatch b) {
    const FwdItem &it = b.it[item_of(b)];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int w = ((int)blockIdx.x - it.blk0) * FWD_WAVES_PER_BLOCK + wv;
    const IT *col = (const IT *)it.col;
    const WT *val = (const WT *)it.val;
    if (it.pair) {
        const int r = it.r0 + 2 * w;
        if (r < it.r1) fwd_ratio_pair(it.row_ptr, col, val, it.a.f, it.a.g, it.a.w, it.a.out, r, it.r1, lane, it.a.eps);
    } else {
        const int r = it.r0 + w;
        if (r < it.r1) fwd_ratio_row(it.row_ptr, col, val, it.a.f, it.a.g, it.a.w, it.a.out, r, lane, it.a.eps);
    }
}

// fused back-projection + SVREM update of each item's pixels
template <typename WT, typename IT>
__global__ void __launch_bounds__(BP_THREADS) k_update_batch(UpdBatch b) {
    const UpdItem &it = b.it[item_of(b)];
    const int gid = ((int)blockIdx.x - it.blk0) * BP_THREADS + threadIdx.x;
    const int n = gid / BP_G, lig = gid % BP_G;
    if (n >= it.N) return;  // whole groups leave together
    update_pixel<UPD_SVREM, WT, IT>(it.ptrT, (const IT *)it.rowT, (const WT *)it.valT, it.sens_t, it.sens, it.N, it.u,
                                    n, lig);
}

// SVREM anchor table of each item: one BP_G-lane group per (subset, pixel)
template <typename WT, typename IT>
__global__ void __launch_bounds__(BP_THREADS) k_anchor_table_batch(AncTabBatch b) {
    const AncTabItem &it = b.it[item_of(b)];
    const int64_t gid = (int64_t)((int)blockIdx.x - it.blk0) * BP_THREADS + threadIdx.x;
    const int64_t q = gid / BP_G;
    const int lig = (int)(gid % BP_G);
    if (q >= (int64_t)it.Ns * it.N) return;  // whole groups leave together
    anchor_entry<UPD_SVREM, WT, IT>(it.ptrT, (const IT *)it.rowT, (const WT *)it.valT, it.row_start, it.Ns, it.N,
                                    it.a, q, lig);
}

// SVREM anchor sums + the first update of each item: a thread per pixel
__global__ void __launch_bounds__(256) k_anchor_sum_batch(AncSumBatch b) {
    const AncSumItem &it = b.it[item_of(b)];
    const int n = ((int)blockIdx.x - it.blk0) * 256 + threadIdx.x;
    if (n >= it.N) return;
    anchor_sum_update_pixel<UPD_SVREM>(it.sens_t, it.sens, it.Ns, it.N, it.a, it.u, n);
}

void add_anchor_table(AncTabBatch &b, const IterPlan &p, const SnapArgs &sa) {
    const Matrix &A = *p.A;
    AncTabItem &it = b.it[b.n++];
    it.ptrT = A.d_ptrT;
    it.rowT = A.d_rowT;
    it.valT = A.d_valT;
    it.row_start = A.d_row_start;
    it.Ns = A.Ns;
    it.N = A.N;
    it.blk0 = b.blocks;
    it.a = sa;
    b.blocks += (int)(((int64_t)A.Ns * A.N * BP_G + BP_THREADS - 1) / BP_THREADS);
}

void add_anchor_sum(AncSumBatch &b, const IterPlan &p, const SnapArgs &sa) {
    const Matrix &A = *p.A;
    AncSumItem &it = b.it[b.n++];
    it.sens_t = A.d_sens_t;
    it.sens = A.d_sens;
    it.Ns = A.Ns;
    it.N = A.N;
    it.blk0 = b.blocks;
    it.a = sa;
    it.u = p.u;
    b.blocks += (A.N + 255) / 256;
}

int launch_anchor_table_batch(const Matrix &types, const AncTabBatch &b, hipStream_t s) {
    if (b.n == 0 || b.blocks == 0) return SVR_OK;
    return with_types(types, [&](auto w, auto i) {
        using WT = decltype(w);
        using IT = decltype(i);
        SVR_HIP(launch_k(k_anchor_table_batch<WT, IT>, b.blocks, BP_THREADS, s, b));
        return SVR_OK;
    });
}

int launch_anchor_sum_batch(const AncSumBatch &b, hipStream_t s) {
    if (b.n == 0 || b.blocks == 0) return SVR_OK;
    SVR_HIP(launch_k(k_anchor_sum_batch, b.blocks, 256, s, b));
    return SVR_OK;
}

void add_forward(FwdBatch &b, const IterPlan &p) {
    const Matrix &A = *p.A;
    FwdItem &it = b.it[b.n++];
    it.row_ptr = A.d_row_ptr;
    it.col = A.d_colt;
    it.val = A.d_val;
    it.a = p.fa;
    it.r0 = p.r0;
    it.r1 = p.r1;
    it.pair = p.pair ? 1 : 0;
    it.blk0 = b.blocks;
    const int64_t rows = p.r1 - p.r0;
    const int64_t waves = p.pair ? (rows + 1) / 2 : rows;
    b.blocks += (int)((waves + FWD_WAVES_PER_BLOCK - 1) / FWD_WAVES_PER_BLOCK);
}

void add_update(UpdBatch &b, const IterPlan &p) {
    const Matrix &A = *p.A;
    UpdItem &it = b.it[b.n++];
    it.ptrT = A.d_ptrT;
    it.rowT = A.d_rowT;
    it.valT = A.d_valT;
    it.sens_t = A.d_sens_t;
    it.sens = A.d_sens;
    it.N = A.N;
    it.blk0 = b.blocks;
    it.u = p.u;
    b.blocks += (int)(((int64_t)A.N * BP_G + BP_THREADS - 1) / BP_THREADS);
}

int launch_forward_batch(const Matrix &types, const FwdBatch &b, hipStream_t s) {
    if (b.n == 0 || b.blocks == 0) return SVR_OK;
    return with_types(types, [&](auto w, auto i) {
        using WT = decltype(w);
        using IT = decltype(i);
        SVR_HIP(launch_k(k_forward_batch<WT, IT>, b.blocks, FWD_THREADS, s, b));
        return SVR_OK;
    });
}

int launch_update_batch(const Matrix &types, const UpdBatch &b, hipStream_t s) {
    if (b.n == 0 || b.blocks == 0) return SVR_OK;
    return with_types(types, [&](auto w, auto i) {
        using WT = decltype(w);
        using IT = decltype(i);
        SVR_HIP(launch_k(k_update_batch<WT, IT>, b.blocks, BP_THREADS, s, b));
        return SVR_OK;
    });
}

}  // namespace svr
