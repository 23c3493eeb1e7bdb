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
    const double b = bp_group(ptrT, rowT, valT, q, u.ratio, lig);
    if (lig != 0) return;
    const float f = u.f[n];
    const PenaltyArgs &p = u.pen;
    float out;
    if (KIND == UPD_OSEM) {
        const float st = sens_t[q];
        out = st > 0.0f ? (float)(((double)f * b) / (double)st) : 0.0f;
    } else if (KIND == UPD_SVREM || KIND == UPD_SEM) {
        const float tau = tau_of(u.Ns, f, b);
        double sh;
        if (KIND == UPD_SVREM)
            sh = (1.0 - u.alpha) * u.s_hat[n] + u.alpha * (((double)tau - (double)u.table[q]) + u.s_anc[n]);
        else
            sh = (1.0 - u.alpha) * u.s_hat[n] + u.alpha * (double)tau;
        u.s_hat[n] = sh;
        double D = 0.0, E = 0.0;
        if (p.beta > 0.0) surrogate_at(u.f, n, p, D, E);
        const double sn = sens[n];
        const double bb = p.beta * D;
        const double cc = (p.beta * (double)f * D + p.beta * E) - sn;
        out = (float)mstep_root(sh, bb, cc, sn);
    } else {
        const float st = sens_t[q];
        const double gr = p.beta > 0.0 ? penalty_grad_at(u.f, n, p) : 0.0;
        double dir;
        double d;
        if (KIND == UPD_SVRG) {
            const float qn = q_of(b, gr, p.beta, u.Ns);
            dir = ((double)qn - (double)u.table[q]) + u.g_tilde[n];
            d = precond_of(u, q, n, f, st);
        } else if (KIND == UPD_SAGA) {
            const float qn = q_of(b, gr, p.beta, u.Ns);
            const float qo = u.table[q];
            const double Qn = u.Q[n];
            dir = ((double)qn - (double)qo) + (Qn - sens[n]) / (double)u.Ns;
            d = precond_of(u, q, n, f, st);
            u.Q[n] = Qn + ((double)qn - (double)qo);
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
    switch (A.wtype) {
        case SVR_W_F32:
            k_update<KIND, float><<<nb, BP_THREADS, 0, s>>>(A.d_ptrT, A.d_rowT, (const float *)A.d_valT,
                                                           A.d_sens_t, A.d_sens, A.N, u);
            break;
        case SVR_W_F16:
            k_update<KIND, _Float16><<<nb, BP_THREADS, 0, s>>>(A.d_ptrT, A.d_rowT, (const _Float16 *)A.d_valT,
                                                              A.d_sens_t, A.d_sens, A.N, u);
            break;
        default:
            k_update<KIND, bf16_t><<<nb, BP_THREADS, 0, s>>>(A.d_ptrT, A.d_rowT, (const bf16_t *)A.d_valT,
                                                            A.d_sens_t, A.d_sens, A.N, u);
    }
    SVR_HIP(hipGetLastError());
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

// ---- snapshot: every subset at the current image -----------------------------
template <int KIND, typename WT>
__global__ void __launch_bounds__(BP_THREADS)
k_snapshot(const int *__restrict__ ptrT, const int *__restrict__ rowT, const WT *__restrict__ valT,
           const int *__restrict__ row_start, const double *__restrict__ sens, int Ns, int N, SnapArgs a) {
    const int gid = blockIdx.x * BP_THREADS + threadIdx.x;
    const int n = gid / BP_G, lig = gid % BP_G;
    if (n >= N) return;
    const float f = a.f[n];
    const PenaltyArgs &p = a.pen;
    double gr = 0.0;
    if (KIND != UPD_SVREM && p.beta > 0.0) gr = penalty_grad_at(a.f, n, p);
    double sum = 0.0;
    for (int t = 0; t < Ns; ++t) {
        const int64_t q = (int64_t)t * N + n;
        const double b = bp_group(ptrT, rowT, valT, q, a.ratio_all + row_start[t], lig);
        float v;
        if (KIND == UPD_SVREM) v = tau_of(Ns, f, b);
        else v = q_of(b, gr, p.beta, Ns);
        if (lig == 0) a.table[q] = v;
        sum = sum + (double)v;
    }
    if (lig != 0) return;
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
static int launch_snapshot_k(const Matrix &A, const SnapArgs &a, hipStream_t s) {
    const int nb = (int)(((int64_t)A.N * BP_G + BP_THREADS - 1) / BP_THREADS);
    switch (A.wtype) {
        case SVR_W_F32:
            k_snapshot<KIND, float><<<nb, BP_THREADS, 0, s>>>(A.d_ptrT, A.d_rowT, (const float *)A.d_valT,
                                                             A.d_row_start, A.d_sens, A.Ns, A.N, a);
            break;
        case SVR_W_F16:
            k_snapshot<KIND, _Float16><<<nb, BP_THREADS, 0, s>>>(A.d_ptrT, A.d_rowT, (const _Float16 *)A.d_valT,
                                                                A.d_row_start, A.d_sens, A.Ns, A.N, a);
            break;
        default:
            k_snapshot<KIND, bf16_t><<<nb, BP_THREADS, 0, s>>>(A.d_ptrT, A.d_rowT, (const bf16_t *)A.d_valT,
                                                              A.d_row_start, A.d_sens, A.Ns, A.N, a);
    }
    SVR_HIP(hipGetLastError());
    return SVR_OK;
}

int launch_snapshot(const Matrix &A, int kind, const SnapArgs &a, hipStream_t s) {
    switch (kind) {
        case UPD_SVREM: return launch_snapshot_k<UPD_SVREM>(A, a, s);
        case UPD_SVRG: return launch_snapshot_k<UPD_SVRG>(A, a, s);
        case UPD_SAGA: return launch_snapshot_k<UPD_SAGA>(A, a, s);
    }
    set_error("snapshot not defined for kind %d", kind);
    return SVR_EINVAL;
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
