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
// Running statistics and table sums are FP64; tables and the iterate FP32.
// The quantities stored in a table at an anchor are computed by the same
// device functions as in the iterations, so they cancel exactly at f = f_anc.
#include <cmath>

#include "common.h"
#include "kernels.h"
#include "penalty.h"

namespace svr {

__device__ inline float tau_of(int Ns, float f, double b) { return (float)(((double)Ns * (double)f) * b); }

__device__ inline float q_of(double b, double gradR, double beta, int Ns) {
    return (float)(b - (beta / (double)Ns) * gradR);
}

__device__ inline double precond_of(const UpdateArgs &u, int64_t q, int n, float f, float st) {
    if (u.dpre) return (double)u.dpre[u.dpre_per_subset ? q : (int64_t)n];
    return st > 0.0f ? (double)f / (double)st : 0.0;
}

template <int KIND, typename WT>
__global__ void __launch_bounds__(BP_THREADS)
k_update(const int *__restrict__ ptrT, const int *__restrict__ rowT, const WT *__restrict__ valT,
         const float *__restrict__ sens_t, const double *__restrict__ sens, int N, UpdateArgs u) {
    const int gid = blockIdx.x * BP_THREADS + threadIdx.x;
    const int n = gid / BP_G, lig = gid % BP_G;
    if (n >= N) return;
    const int64_t q = (int64_t)u.t * N + n;
    const PenaltyArgs &p = u.pen;
    // per-pixel operands first: they do not depend on the gather below, so
    // their loads overlap with it
    const float f = u.f[n];
    constexpr bool EM = (KIND == UPD_SVREM || KIND == UPD_SEM);
    const float st = (KIND != UPD_SVREM && KIND != UPD_SEM) ? sens_t[q] : 0.0f;
    const double sh0 = EM ? u.s_hat[n] : 0.0;
    const float tab = (KIND == UPD_SVREM || KIND == UPD_SVRG || KIND == UPD_SAGA) ? u.table[q] : 0.0f;
    const double sanc = (KIND == UPD_SVREM) ? u.s_anc[n] : 0.0;
    const double sn = (EM || KIND == UPD_SAGA) ? sens[n] : 0.0;
    const double gt = (KIND == UPD_SVRG) ? u.g_tilde[n] : 0.0;
    const double Qn = (KIND == UPD_SAGA) ? u.Q[n] : 0.0;
    double D = 0.0, E = 0.0, gr = 0.0;
    if (lig == 0 && p.beta > 0.0) {
        if (EM) surrogate_at(u.f, n, p, D, E);
        else if (KIND != UPD_OSEM) gr = penalty_grad_at(u.f, n, p);
    }
    const double b = bp_group(ptrT, rowT, valT, q, u.ratio, lig);
    if (lig != 0) return;
    float out;
    if (KIND == UPD_OSEM) {
        out = st > 0.0f ? (float)(((double)f * b) / (double)st) : 0.0f;
    } else if (EM) {
        const float tau = tau_of(u.Ns, f, b);
        double sh;
        if (KIND == UPD_SVREM)
            sh = (1.0 - u.alpha) * sh0 + u.alpha * (((double)tau - (double)tab) + sanc);
        else
            sh = (1.0 - u.alpha) * sh0 + u.alpha * (double)tau;
        u.s_hat[n] = sh;
        const double bb = p.beta * D;
        const double cc = (p.beta * (double)f * D + p.beta * E) - sn;
        out = (float)mstep_root(sh, bb, cc, sn);
    } else {
        double dir, d;
        if (KIND == UPD_SVRG) {
            const float qn = q_of(b, gr, p.beta, u.Ns);
            dir = ((double)qn - (double)tab) + gt;
            d = precond_of(u, q, n, f, st);
        } else if (KIND == UPD_SAGA) {
            const float qn = q_of(b, gr, p.beta, u.Ns);
            dir = ((double)qn - (double)tab) + (Qn - sn) / (double)u.Ns;
            d = precond_of(u, q, n, f, st);
            u.Q[n] = Qn + ((double)qn - (double)tab);
            u.table[q] = qn;
        } else {  // SGA / BSREM: iteration-dependent subset preconditioner
            dir = (b - (double)st) - (p.beta / (double)u.Ns) * gr;
            d = st > 0.0f ? (double)f / (double)st : 0.0;
        }
        out = (float)fmax(0.0, (double)f + (u.alpha * d) * dir);
    }
    u.f_out[n] = out;
}

template <int KIND>
static int launch_update_k(const Matrix &A, const UpdateArgs &u, hipStream_t s) {
    const int nb = (int)(((int64_t)A.N * BP_G + BP_THREADS - 1) / BP_THREADS);
    hipError_t e;
    switch (A.wtype) {
        case SVR_W_F32:
            e = launch_k(k_update<KIND, float>, nb, BP_THREADS, s, A.d_ptrT, A.d_rowT, (const float *)A.d_valT,
                         A.d_sens_t, A.d_sens, A.N, u);
            break;
        case SVR_W_F16:
            e = launch_k(k_update<KIND, _Float16>, nb, BP_THREADS, s, A.d_ptrT, A.d_rowT,
                         (const _Float16 *)A.d_valT, A.d_sens_t, A.d_sens, A.N, u);
            break;
        default:
            e = launch_k(k_update<KIND, bf16_t>, nb, BP_THREADS, s, A.d_ptrT, A.d_rowT, (const bf16_t *)A.d_valT,
                         A.d_sens_t, A.d_sens, A.N, u);
    }
    SVR_HIP(e);
    return SVR_OK;
}

int launch_update(const Matrix &A, int kind, const UpdateArgs &u, hipStream_t s) {
    switch (kind) {
        case UPD_OSEM: return launch_update_k<UPD_OSEM>(A, u, s);
        case UPD_SVREM: return launch_update_k<UPD_SVREM>(A, u, s);
        case UPD_SVRG: return launch_update_k<UPD_SVRG>(A, u, s);
        case UPD_SAGA: return launch_update_k<UPD_SAGA>(A, u, s);
        case UPD_SGA: return launch_update_k<UPD_SGA>(A, u, s);
        case UPD_SEM: return launch_update_k<UPD_SEM>(A, u, s);
    }
    set_error("unknown update kind %d", kind);
    return SVR_EINVAL;
}

// ---- anchor pass ---------------------------------------------------------------
// table kernel: one BP_G-lane group per (subset, pixel), the same gather and
// the same tau / q expressions as the iteration kernel
template <int KIND, typename WT>
__global__ void __launch_bounds__(BP_THREADS)
k_anchor_table(const int *__restrict__ ptrT, const int *__restrict__ rowT, const WT *__restrict__ valT,
               const int *__restrict__ row_start, int Ns, int N, SnapArgs a) {
    const int64_t gid = (int64_t)blockIdx.x * BP_THREADS + threadIdx.x;
    const int64_t q = gid / BP_G;
    const int lig = (int)(gid % BP_G);
    if (q >= (int64_t)Ns * N) return;
    const int t = (int)(q / N), n = (int)(q - (int64_t)t * N);
    const float f = a.f[n];
    const PenaltyArgs &p = a.pen;
    double gr = 0.0;
    if (KIND != UPD_SVREM && lig == 0 && p.beta > 0.0) gr = penalty_grad_at(a.f, n, p);
    const double b = bp_group(ptrT, rowT, valT, q, a.ratio_all + row_start[t], lig);
    if (lig != 0) return;
    a.table[q] = (KIND == UPD_SVREM) ? tau_of(Ns, f, b) : q_of(b, gr, p.beta, Ns);
}

// sum kernel: FP64 sums over t in increasing order
template <int KIND>
__global__ void __launch_bounds__(256)
k_anchor_sum(const double *__restrict__ sens, int Ns, int N, SnapArgs a) {
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    double sum = 0.0;
    for (int t = 0; t < Ns; ++t) sum = sum + (double)a.table[(int64_t)t * N + n];
    if (KIND == UPD_SVREM) {
        const double sa = sum / (double)Ns;
        a.s_anc[n] = sa;
        if (a.init_shat) a.s_hat[n] = sa;
    } else if (KIND == UPD_SVRG) {
        a.g_tilde[n] = (sum - sens[n]) / (double)Ns;
    } else {
        a.Q[n] = sum;
    }
}

template <int KIND>
static int launch_anchor_table_k(const Matrix &A, const SnapArgs &a, hipStream_t s) {
    const int nb = (int)(((int64_t)A.Ns * A.N * BP_G + BP_THREADS - 1) / BP_THREADS);
    hipError_t e;
    switch (A.wtype) {
        case SVR_W_F32:
            e = launch_k(k_anchor_table<KIND, float>, nb, BP_THREADS, s, A.d_ptrT, A.d_rowT,
                         (const float *)A.d_valT, A.d_row_start, A.Ns, A.N, a);
            break;
        case SVR_W_F16:
            e = launch_k(k_anchor_table<KIND, _Float16>, nb, BP_THREADS, s, A.d_ptrT, A.d_rowT,
                         (const _Float16 *)A.d_valT, A.d_row_start, A.Ns, A.N, a);
            break;
        default:
            e = launch_k(k_anchor_table<KIND, bf16_t>, nb, BP_THREADS, s, A.d_ptrT, A.d_rowT,
                         (const bf16_t *)A.d_valT, A.d_row_start, A.Ns, A.N, a);
    }
    SVR_HIP(e);
    return SVR_OK;
}

int launch_anchor_table(const Matrix &A, int kind, const SnapArgs &a, hipStream_t s) {
    switch (kind) {
        case UPD_SVREM: return launch_anchor_table_k<UPD_SVREM>(A, a, s);
        case UPD_SVRG: return launch_anchor_table_k<UPD_SVRG>(A, a, s);
        case UPD_SAGA: return launch_anchor_table_k<UPD_SAGA>(A, a, s);
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
        default: set_error("no anchor pass for kind %d", kind); return SVR_EINVAL;
    }
    SVR_HIP(e);
    return SVR_OK;
}

// ---- frozen preconditioner --------------------------------------------------
__global__ void k_precond(const float *f0, const float *sens_t, const double *sens, int Ns, int N,
                          int per_subset, float *d) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (per_subset) {
        if (i >= (int64_t)Ns * N) return;
        const int n = (int)(i % N);
        const float st = sens_t[i];
        d[i] = st > 0.0f ? (float)((double)f0[n] / (double)st) : 0.0f;
    } else {
        if (i >= N) return;
        d[i] = sens[i] > 0.0 ? (float)((double)f0[i] / sens[i]) : 0.0f;
    }
}

int launch_precond(const Matrix &A, const float *f0, int per_subset, float *d, hipStream_t s) {
    const int64_t n = per_subset ? (int64_t)A.Ns * A.N : A.N;
    k_precond<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(f0, A.d_sens_t, A.d_sens, A.Ns, A.N, per_subset, d);
    SVR_HIP(hipGetLastError());
    return SVR_OK;
}

}  // namespace svr
