// Fused back-projection + per-pixel update kernels.
//
// One group of BP_G lanes per pixel gathers b_n = (A_t^T r)_n over the
// pixel's transposed row of subset t, then the group's first lane applies
// the algorithm's update with the penalty stencil fused in:
//   OSEM  (Sec. 2.2, eq. Mstep)          f+ = f b / (A_t^T 1)
//   SVREM (Sec. 2.3 eq. tempsvrem + Sec. 3 eq. svrsurder)
//         tau = Ns f b;  s_hat <- (1-a) s_hat + a (tau - tau_anc_t + s_anc);
//         f+ = root(s_hat, beta sum d, beta f sum d + beta sum d f_j - A^T 1)
//   SVRG  (Sec. 4, eq. svrg_update)       q = b - beta/Ns grad R(f);
//         f+ = max(0, f + a d (q - q_anc_t + g_tilde))
//   SAGA  (Sec. 4, eq. saga_update)       f+ = max(0, f + a d (q - q_t + (Q - A^T 1)/Ns));
//         Q += q - q_t; q_t = q
//   SGA / BSREM (Sec. 4 eq. sga, Sec. 5.1) f+ = max(0, f + a (f / A_t^T 1) (b - A_t^T 1 - beta/Ns grad R))
//   SEM   (Sec. 2.3, eq. tempsem)         s_hat <- (1-a) s_hat + a tau; f+ = root(...)
//   SAGA-EM (Sec. 2.3, remark after eq. tempsvrem)
//         s_hat <- (1-a) s_hat + a (tau_t - S_t + Q/Ns); S_t2 <- tau_t2; f+ = root(...)
// Running statistics and table sums are FP64; tables and the iterate FP32.
// The quantities stored in a table at an anchor are computed by the same
// back-projection and update expressions as in the iterations; the iteration
// that takes the anchor uses the table entry itself (anchor_sum_update_pixel),
// so its anchor terms cancel exactly.
#include <cmath>

#include "common.h"
#include "kernels.h"
#include "penalty.h"
#include "phases.h"

namespace svr {

// One BP_G-lane group per pixel, 64 consecutive pixels per workgroup; XCD x
// takes a contiguous eighth of the image (xcd_chunk), so the transposed-row
// lines two neighbouring workgroups share, the stencil's neighbour rows and
// the 4 x 8 tiles of the tiled write stay in one L2 (HBM counters: 1.17x ->
// 1.03x of the algorithmic bytes)
template <int KIND, typename WT, typename IT, int U>
__global__ void __launch_bounds__(BP_THREADS)
k_update(const int *__restrict__ ptrT, const IT *__restrict__ rowT, const WT *__restrict__ valT,
         const float *__restrict__ sens_t, const double *__restrict__ sens, int N, int per, UpdateArgs u) {
    const int gid = xcd_chunk(blockIdx.x, per) * BP_THREADS + threadIdx.x;
    const int n = gid / BP_G, lig = gid % BP_G;
    if (n >= N) return;
    update_pixel<KIND, WT, IT, U>(ptrT, rowT, valT, sens_t, sens, N, u, n, lig);
}

// the update with U index/weight loads per lane and batch (the tuned width,
// else BP_U); the width changes neither the entries a lane adds nor their
// order, so the result is bitwise the same for every U
template <int KIND, int U>
static int launch_update_u(const Matrix &A, const UpdateArgs &u, hipStream_t s) {
    int per = 0;
    const int nb = xcd_grid(((int64_t)A.N * BP_G + BP_THREADS - 1) / BP_THREADS, per);
    return with_types(A, [&](auto w, auto i) {
        using WT = decltype(w);
        using IT = decltype(i);
        SVR_HIP(launch_k(k_update<KIND, WT, IT, U>, nb, BP_THREADS, s, A.d_ptrT, (const IT *)A.d_rowT,
                         (const WT *)A.d_valT, A.d_sens_t, A.d_sens, A.N, per, u));
        return SVR_OK;
    });
}

template <int KIND>
static int launch_update_k(const Matrix &A, const UpdateArgs &u, hipStream_t s) {
    switch (A.sub_bp_u) {
        case 3: return launch_update_u<KIND, 3>(A, u, s);
        case 4: return launch_update_u<KIND, 4>(A, u, s);
        case 6: return launch_update_u<KIND, 6>(A, u, s);
        case 8: return launch_update_u<KIND, 8>(A, u, s);
        default: return launch_update_u<KIND, BP_U>(A, u, s);
    }
}

int launch_update(const Matrix &A, int kind, const UpdateArgs &u, hipStream_t s) {
    switch (kind) {
        case UPD_OSEM: return launch_update_k<UPD_OSEM>(A, u, s);
        case UPD_SVREM: return launch_update_k<UPD_SVREM>(A, u, s);
        case UPD_SVRG: return launch_update_k<UPD_SVRG>(A, u, s);
        case UPD_SAGA: return launch_update_k<UPD_SAGA>(A, u, s);
        case UPD_SGA: return launch_update_k<UPD_SGA>(A, u, s);
        case UPD_SEM: return launch_update_k<UPD_SEM>(A, u, s);
        case UPD_SAGAEM: return launch_update_k<UPD_SAGAEM>(A, u, s);
    }
    set_error("unknown update kind %d", kind);
    return SVR_EINVAL;
}

// ---- anchor pass ---------------------------------------------------------------
__global__ void __launch_bounds__(256) k_penalty_grad(const float *__restrict__ f, int N, PenaltyArgs p,
                                                      double *__restrict__ out) {
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    out[n] = penalty_grad_at(f, n, p);
}

int launch_penalty_grad(const Matrix &A, const float *f, const PenaltyArgs &p, double *out, hipStream_t s) {
    SVR_HIP(launch_k(k_penalty_grad, (A.N + 255) / 256, 256, s, f, A.N, p, out));
    return SVR_OK;
}

// table kernel: one BP_G-lane group per (subset, pixel), the same gather and
// the same tau / q expressions as the iteration kernel
template <int KIND, typename WT, typename IT>
__global__ void __launch_bounds__(BP_THREADS)
k_anchor_table(const int *__restrict__ ptrT, const IT *__restrict__ rowT, const WT *__restrict__ valT,
               const int *__restrict__ row_start, int Ns, int N, SnapArgs a) {
    const int64_t gid = (int64_t)blockIdx.x * BP_THREADS + threadIdx.x;
    const int64_t q = gid / BP_G;
    const int lig = (int)(gid % BP_G);
    if (q >= (int64_t)Ns * N) return;
    anchor_entry<KIND, WT, IT>(ptrT, rowT, valT, row_start, Ns, N, a, q, lig);
}

// The same table with runs: each wavefront owns `steps` x (64 / BP_G)
// consecutive (subset, pixel) rows; at step i its groups take the next
// 64 / BP_G rows, pipelined by bp_run.
template <int KIND, typename WT, typename IT>
__global__ void __launch_bounds__(BP_THREADS)
k_anchor_table_run(const int *__restrict__ ptrT, const IT *__restrict__ rowT, const WT *__restrict__ valT,
               const int *__restrict__ row_start, int Ns, int N, int steps, SnapArgs a) {
    constexpr int GPW = 64 / BP_G;  // groups per wavefront
    const int lane = threadIdx.x & 63, gi = lane / BP_G, lig = lane % BP_G;
    const int64_t wave = ((int64_t)blockIdx.x * BP_THREADS + threadIdx.x) >> 6;
    const int64_t total = (int64_t)Ns * N;  // < 2^31
    const int64_t q0 = wave * GPW * steps + gi;
    bp_run<WT, IT>(ptrT, rowT, valT, steps, lig, a.ratio_all,
                   [&](int i, int64_t &q, const float *&y, float &f) {
                       q = q0 + (int64_t)GPW * i;
                       if (q >= total) return false;
                       const int t = (int)q / N;
                       y = a.ratio_all + row_start[t];
                       f = a.f[(int)q - t * N];
                       return true;
                   },
                   [&](int i, double b, float f) {
                       const int64_t q = q0 + (int64_t)GPW * i;
                       if (lig != 0 || q >= total) return;
                       anchor_finish<KIND>(a, Ns, q, (int)q % N, f, b);
                   });
}

// (subset, pixel) rows per lane group of a whole-table pass.  Without a
// tuned value: 1 (the run kernel holds two rows' operands in registers,
// which costs occupancy; svr_matrix_tune measures whether runs pay off)
int table_run_length(const Matrix &A) {
    if (A.run_bp > 0) return std::min(A.run_bp, 1024);
    return 1;
}

template <int KIND>
__global__ void __launch_bounds__(256)
k_anchor_sum(const double *__restrict__ sens, int Ns, int N, SnapArgs a) {
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    anchor_sum_pixel<KIND>(sens, Ns, N, a, n);
}

template <int KIND>
__global__ void __launch_bounds__(256)
k_anchor_sum_update(const float *__restrict__ sens_t, const double *__restrict__ sens, int Ns, int N, SnapArgs a,
                    UpdateArgs u) {
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    anchor_sum_update_pixel<KIND>(sens_t, sens, Ns, N, a, u, n);
}

int launch_anchor_sum_update(const Matrix &A, int kind, const SnapArgs &a, const UpdateArgs &u, hipStream_t s) {
    const int nb = (A.N + 255) / 256;
    hipError_t e;
    switch (kind) {
        case UPD_SVREM:
            e = launch_k(k_anchor_sum_update<UPD_SVREM>, nb, 256, s, A.d_sens_t, A.d_sens, A.Ns, A.N, a, u);
            break;
        case UPD_SVRG:
            e = launch_k(k_anchor_sum_update<UPD_SVRG>, nb, 256, s, A.d_sens_t, A.d_sens, A.Ns, A.N, a, u);
            break;
        case UPD_SAGA:
            e = launch_k(k_anchor_sum_update<UPD_SAGA>, nb, 256, s, A.d_sens_t, A.d_sens, A.Ns, A.N, a, u);
            break;
        case UPD_SAGAEM:
            e = launch_k(k_anchor_sum_update<UPD_SAGAEM>, nb, 256, s, A.d_sens_t, A.d_sens, A.Ns, A.N, a, u);
            break;
        default: set_error("no anchor pass for kind %d", kind); return SVR_EINVAL;
    }
    SVR_HIP(e);
    return SVR_OK;
}

template <int KIND>
static int launch_anchor_table_k(const Matrix &A, const SnapArgs &a, hipStream_t s) {
    constexpr int GPW = 64 / BP_G;
    const int steps = table_run_length(A);
    const int64_t waves = ((int64_t)A.Ns * A.N + (int64_t)GPW * steps - 1) / ((int64_t)GPW * steps);
    const int nb = (int)((waves * 64 + BP_THREADS - 1) / BP_THREADS);
    return with_types(A, [&](auto w, auto i) {
        using WT = decltype(w);
        using IT = decltype(i);
        if (steps == 1)
            SVR_HIP(launch_k(k_anchor_table<KIND, WT, IT>, nb, BP_THREADS, s, A.d_ptrT, (const IT *)A.d_rowT,
                             (const WT *)A.d_valT, A.d_row_start, A.Ns, A.N, a));
        else
            SVR_HIP(launch_k(k_anchor_table_run<KIND, WT, IT>, nb, BP_THREADS, s, A.d_ptrT, (const IT *)A.d_rowT,
                             (const WT *)A.d_valT, A.d_row_start, A.Ns, A.N, steps, a));
        return SVR_OK;
    });
}

int launch_anchor_table(const Matrix &A, int kind, const SnapArgs &a, hipStream_t s) {
    switch (kind) {
        case UPD_SVREM: return launch_anchor_table_k<UPD_SVREM>(A, a, s);
        case UPD_SVRG: return launch_anchor_table_k<UPD_SVRG>(A, a, s);
        case UPD_SAGA: return launch_anchor_table_k<UPD_SAGA>(A, a, s);
        case UPD_SAGAEM: return launch_anchor_table_k<UPD_SAGAEM>(A, a, s);
    }
    set_error("no anchor pass for kind %d", kind);
    return SVR_EINVAL;
}

int launch_anchor_sum(const Matrix &A, int kind, const SnapArgs &a, hipStream_t s) {
    const int nb = (A.N + 255) / 256;
    hipError_t e;
    switch (kind) {
        case UPD_SVREM: e = launch_k(k_anchor_sum<UPD_SVREM>, nb, 256, s, A.d_sens, A.Ns, A.N, a); break;
        case UPD_SVRG: e = launch_k(k_anchor_sum<UPD_SVRG>, nb, 256, s, A.d_sens, A.Ns, A.N, a); break;
        case UPD_SAGA: e = launch_k(k_anchor_sum<UPD_SAGA>, nb, 256, s, A.d_sens, A.Ns, A.N, a); break;
        case UPD_SAGAEM: e = launch_k(k_anchor_sum<UPD_SAGAEM>, nb, 256, s, A.d_sens, A.Ns, A.N, a); break;
        default: set_error("no anchor pass for kind %d", kind); return SVR_EINVAL;
    }
    SVR_HIP(e);
    return SVR_OK;
}

// ---- frozen preconditioner --------------------------------------------------
__global__ void k_precond(const float *f0, const float *sens_t, const double *sens, int Ns, int N,
                          int per_subset, float *d) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (per_subset ? (int64_t)Ns * N : (int64_t)N)) return;
    precond_entry(f0, sens_t, sens, N, per_subset, i, d);
}

int launch_precond(const Matrix &A, const float *f0, int per_subset, float *d, hipStream_t s) {
    const int64_t n = per_subset ? (int64_t)A.Ns * A.N : A.N;
    k_precond<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(f0, A.d_sens_t, A.d_sens, A.Ns, A.N, per_subset, d);
    SVR_HIP(hipGetLastError());
    return SVR_OK;
}

}  // namespace svr
