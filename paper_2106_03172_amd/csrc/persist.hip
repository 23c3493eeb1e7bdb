// Persistent epoch kernel: one cooperative launch runs a whole epoch call
// (every anchor pass, subset forward projection and fused update of the
// given subset sequence), with grid-wide barriers between the phases in
// place of kernel boundaries.
//
// Each subset update has two grid-wide dependencies: every pixel's gather
// needs every ratio of the subset, and every ray of the next subset needs
// every updated pixel.  With one kernel per phase each dependency costs a
// kernel launch and ramp; here it costs one barrier.  The phases call the
// same device functions as the one-kernel-per-phase path, so both paths
// compute bitwise the same values.
//
// Barrier: blocks arrive on one of 8 sub-counters (blockIdx % 8), the last
// arrival of each sub-counter arrives on a top counter, and the last top
// arrival resets the counters and advances a generation word that every
// block polls.  Agent-scope release/acquire fences around it make the
// phase's global writes visible across XCDs.  The poll is bounded: a block
// that waits longer than SPIN_LIMIT polls raises an abort flag, every block
// then leaves the kernel, and the host reports the failure.
#include <cmath>

#include "common.h"
#include "kernels.h"
#include "penalty.h"
#include "phases.h"

namespace svr {

constexpr int PT_THREADS = 1024;                  // 16 wavefronts per block
constexpr unsigned SYNC_STRIDE = 32;              // words between counters (128 B)
constexpr unsigned SYNC_TOP = 8 * SYNC_STRIDE;
constexpr unsigned SYNC_GEN = 9 * SYNC_STRIDE;
constexpr unsigned SYNC_ABORT = 10 * SYNC_STRIDE;
constexpr unsigned SPIN_LIMIT = 1u << 22;         // ~ seconds of polling

__device__ inline bool grid_barrier(unsigned *gs, unsigned &gen_local, int *abort_lds) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned nb = gridDim.x;
        const unsigned g = gen_local;
        int abort = 0;
        __threadfence();  // release this block's writes of the phase
        const unsigned grp = blockIdx.x & 7u;
        const unsigned in_grp = (nb - grp + 7u) / 8u;
        const unsigned ngrp = nb < 8u ? nb : 8u;
        const unsigned prev = __hip_atomic_fetch_add(&gs[grp * SYNC_STRIDE], 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        if (prev == in_grp - 1u) {
            __hip_atomic_store(&gs[grp * SYNC_STRIDE], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned p2 = __hip_atomic_fetch_add(&gs[SYNC_TOP], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (p2 == ngrp - 1u) {
                __hip_atomic_store(&gs[SYNC_TOP], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&gs[SYNC_GEN], g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        unsigned spins = 0;
        while (__hip_atomic_load(&gs[SYNC_GEN], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
            if (__hip_atomic_load(&gs[SYNC_ABORT], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                abort = 1;
                break;
            }
            if (++spins > SPIN_LIMIT) {
                __hip_atomic_store(&gs[SYNC_ABORT], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                abort = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __threadfence();  // acquire the other blocks' writes
        gen_local = g + 1u;
        *abort_lds = abort;
    }
    __syncthreads();
    return *abort_lds == 0;
}

template <int KIND, typename WT, typename IT>
__global__ void __launch_bounds__(PT_THREADS) k_epoch(EpochArgs e) {
    __shared__ int abort_lds;
    const WT *val = (const WT *)e.val;
    const WT *valT = (const WT *)e.valT;
    const IT *col = (const IT *)e.col;
    const IT *rowT = (const IT *)e.rowT;
    const int nthreads = gridDim.x * blockDim.x;
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int gwave = gtid >> 6, nwaves = nthreads >> 6;
    const int ggroup = gtid / BP_G, ngroups = nthreads / BP_G, lig = gtid % BP_G;
    const int N = e.N, Ns = e.Ns;
    unsigned gen = 0;
    int cur = e.cur0;
    const bool vr_anchor = (KIND == UPD_SVREM || KIND == UPD_SVRG);
    for (int i = 0; i < e.n; ++i) {
        const int t = e.order[i];
        const long long k = e.k0 + i;
        const float *f = cur ? e.f1 : e.f0;
        float *fo = cur ? e.f0 : e.f1;
        const bool anchor = vr_anchor ? (k % ((long long)e.eta * Ns) == 0) : (KIND == UPD_SAGA && k == 0);
        if (anchor) {
            if (forward_pairs_for(e.M, e.pair_rows)) {
                for (int r = 2 * gwave; r < e.M; r += 2 * nwaves)
                    fwd_ratio_pair(e.row_ptr, col, val, e.ft, e.g, e.w, e.ratio, r, e.M, lane, e.eps);
            } else {
                for (int r = gwave; r < e.M; r += nwaves)
                    fwd_ratio_row(e.row_ptr, col, val, e.ft, e.g, e.w, e.ratio, r, lane, e.eps);
            }
            if (!grid_barrier(e.sync, gen, &abort_lds)) goto aborted;
            SnapArgs sa{};
            sa.ratio_all = e.ratio;
            sa.f = f;
            sa.table = e.table;
            sa.s_anc = e.s_anc;
            sa.s_hat = e.s_hat;
            sa.init_shat = (k == 0) || (e.flags & SVR_FLAG_RESET_SHAT_AT_ANCHOR);
            sa.g_tilde = e.g_tilde;
            sa.Q = e.Q;
            sa.pen = e.pen;
            for (long long q = ggroup; q < (long long)Ns * N; q += ngroups)
                anchor_entry<KIND, WT, IT>(e.ptrT, rowT, valT, e.row_start, Ns, N, sa, q, lig);
            if (!grid_barrier(e.sync, gen, &abort_lds)) goto aborted;
            for (int n = gtid; n < N; n += nthreads) anchor_sum_pixel<KIND>(e.sens, Ns, N, sa, n);
            if (!grid_barrier(e.sync, gen, &abort_lds)) goto aborted;
        }
        if ((KIND == UPD_SVRG || KIND == UPD_SAGA) && k == 0 && e.dpre) {
            const long long nd = e.dpre_per_subset ? (long long)Ns * N : (long long)N;
            for (long long q = gtid; q < nd; q += nthreads)
                precond_entry(f, e.sens_t, e.sens, N, e.dpre_per_subset, q, e.dpre);
            if (!grid_barrier(e.sync, gen, &abort_lds)) goto aborted;
        }
        {
            const int r0 = e.row_start[t], r1 = e.row_start[t + 1];
            if (forward_pairs_for(r1 - r0, e.pair_rows)) {
                for (int r = r0 + 2 * gwave; r < r1; r += 2 * nwaves)
                    fwd_ratio_pair(e.row_ptr, col, val, e.ft, e.g, e.w, e.ratio, r, r1, lane, e.eps);
            } else {
                for (int r = r0 + gwave; r < r1; r += nwaves)
                    fwd_ratio_row(e.row_ptr, col, val, e.ft, e.g, e.w, e.ratio, r, lane, e.eps);
            }
            if (!grid_barrier(e.sync, gen, &abort_lds)) goto aborted;
            UpdateArgs u{};
            u.t = t;
            u.Ns = Ns;
            u.ratio = e.ratio + r0;
            u.f = f;
            u.f_out = fo;
            u.ft_out = e.ft;
            u.tx = e.tx;
            u.alpha = e.decaying ? e.alpha / (e.decay * (double)k + 1.0) : e.alpha;
            u.s_hat = e.s_hat;
            u.s_anc = e.s_anc;
            u.table = e.table;
            u.Q = e.Q;
            u.g_tilde = e.g_tilde;
            u.dpre = e.dpre;
            u.dpre_per_subset = e.dpre_per_subset;
            u.shat_zero = (KIND == UPD_SEM && k == 0);
            u.pen = e.pen;
            for (int n = ggroup; n < N; n += ngroups)
                update_pixel<KIND, WT, IT>(e.ptrT, rowT, valT, e.sens_t, e.sens, N, u, n, lig);
            if (!grid_barrier(e.sync, gen, &abort_lds)) goto aborted;
        }
        cur ^= 1;
    }
    return;
aborted:
    if (gtid == 0) e.status[0] = 1;
}

template <int KIND, typename WT, typename IT>
static int launch_epoch_t(const EpochArgs &e, hipStream_t s, int *grid_cache) {
    auto kern = k_epoch<KIND, WT, IT>;
    if (*grid_cache <= 0) {
        int dev = 0, cus = 0, per_cu = 0;
        SVR_HIP(hipGetDevice(&dev));
        SVR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        SVR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, PT_THREADS, 0));
        if (per_cu < 1) {
            set_error("persistent epoch kernel does not fit on a compute unit");
            return SVR_EDEVICE;
        }
        *grid_cache = cus * std::min(per_cu, 2);
    }
    EpochArgs a = e;
    void *args[] = {&a};
    LaunchEvents &tm = pending_timing();
    if (tm.start) SVR_HIP(hipEventRecord(tm.start, s));
    SVR_HIP(hipLaunchCooperativeKernel((const void *)kern, dim3(*grid_cache), dim3(PT_THREADS), args, 0, s));
    if (tm.start) {
        SVR_HIP(hipEventRecord(tm.stop, s));
        tm.start = tm.stop = nullptr;
    }
    return SVR_OK;
}

template <int KIND>
static int launch_epoch_k(const Matrix &A, const EpochArgs &e, hipStream_t s, int *grid_cache) {
    return with_types(A, [&](auto w, auto i) {
        return launch_epoch_t<KIND, decltype(w), decltype(i)>(e, s, grid_cache);
    });
}

int launch_epoch(const Matrix &A, int kind, const EpochArgs &e, hipStream_t s, int *grid_cache) {
    switch (kind) {
        case UPD_OSEM: return launch_epoch_k<UPD_OSEM>(A, e, s, grid_cache);
        case UPD_SVREM: return launch_epoch_k<UPD_SVREM>(A, e, s, grid_cache);
        case UPD_SVRG: return launch_epoch_k<UPD_SVRG>(A, e, s, grid_cache);
        case UPD_SAGA: return launch_epoch_k<UPD_SAGA>(A, e, s, grid_cache);
        case UPD_SGA: return launch_epoch_k<UPD_SGA>(A, e, s, grid_cache);
        case UPD_SEM: return launch_epoch_k<UPD_SEM>(A, e, s, grid_cache);
    }
    set_error("unknown update kind %d", kind);
    return SVR_EINVAL;
}

int persistent_sync_words() { return 11 * (int)SYNC_STRIDE; }

}  // namespace svr
