// Per-pixel and per-(subset, pixel) bodies of the fused update and anchor
// kernels, shared by the one-kernel-per-phase path (update.hip), the
// persistent epoch kernel (persist.hip) and the batched serving kernels
// (batch.hip), so all of them compute bitwise the same.
#pragma once

#include "common.h"
#include "kernels.h"
#include "penalty.h"

namespace svr {

__device__ inline float tau_of(int Ns, float f, double b) { return (float)(((double)Ns * (double)f) * b); }

__device__ inline float q_of(double b, double gradR, double beta, int Ns) {
    return (float)(b - (beta / (double)Ns) * gradR);
}

// OSEM update of one pixel (Sec. 2.2, eq. Mstep)
__device__ inline float osem_math(float f, double b, float st) {
    return st > 0.0f ? (float)(((double)f * b) / (double)st) : 0.0f;
}

// SVREM statistic recursion (Sec. 2.3, eq. tempsvrem) and penalised M-step
// (Sec. 3): returns f+ and the new running statistic in *sh_out
__device__ inline float svrem_math_tau(double alpha, double beta, float f, float tau, double sh0, float tab,
                                       double sanc, double sn, double D, double E, double *sh_out) {
    const double sh = (1.0 - alpha) * sh0 + alpha * (((double)tau - (double)tab) + sanc);
    *sh_out = sh;
    const double bb = beta * D;
    const double cc = (beta * (double)f * D + beta * E) - sn;
    return (float)mstep_root(sh, bb, cc, sn);
}

__device__ inline float svrem_math(int Ns, double alpha, double beta, float f, double b, double sh0, float tab,
                                   double sanc, double sn, double D, double E, double *sh_out) {
    return svrem_math_tau(alpha, beta, f, tau_of(Ns, f, b), sh0, tab, sanc, sn, D, E, sh_out);
}

__device__ inline double precond_of(const UpdateArgs &u, int64_t q, int n, float f, float st) {
    if (u.dpre) return (double)u.dpre[u.dpre_per_subset ? q : (int64_t)n];
    return st > 0.0f ? (double)f / (double)st : 0.0;
}

// One pixel's fused back-projection and update; the BP_G lanes of the
// pixel's group call it together; U index/weight loads per lane and batch.
template <int KIND, typename WT, typename IT, int U = BP_U>
__device__ inline void update_pixel(const int *__restrict__ ptrT, const IT *__restrict__ rowT,
                                    const WT *__restrict__ valT, const float *__restrict__ sens_t,
                                    const double *__restrict__ sens, int N, const UpdateArgs &u, int n, int lig) {
    const int64_t q = (int64_t)u.t * N + n;
    const PenaltyArgs &p = u.pen;
    // The transposed row's bounds first (the gather chain starts there), then
    // every per-pixel operand and the stencil's neighbour values: none of
    // them depends on the gather, so all their loads are in flight with it;
    // the penalty's stencil sums run while the gather's first batch is.
    const int beg = ptrT[q], end = ptrT[q + 1];
    const int iy = n / p.nx, ix = n - iy * p.nx;
    const float f = u.f[n];
    constexpr bool EM = (KIND == UPD_SVREM || KIND == UPD_SEM || KIND == UPD_SAGAEM);
    const float st = !EM ? sens_t[q] : 0.0f;
    const double sh_ld = EM ? u.s_hat[n] : 0.0;  // loaded unconditionally, selected below
    const double sh0 = u.shat_zero ? 0.0 : sh_ld;
    const float tab = (KIND == UPD_SVREM || KIND == UPD_SVRG || KIND == UPD_SAGA || KIND == UPD_SAGAEM) ? u.table[q]
                                                                                                      : 0.0f;
    const double sanc = (KIND == UPD_SVREM) ? u.s_anc[n] : 0.0;
    const double sn = (EM || KIND == UPD_SAGA) ? sens[n] : 0.0;
    const double gt = (KIND == UPD_SVRG) ? u.g_tilde[n] : 0.0;
    const double Qn = (KIND == UPD_SAGA || KIND == UPD_SAGAEM) ? u.Q[n] : 0.0;
    // SAGA-EM: the refreshed subset's table entry (its own gather below when t2 != t)
    const int64_t q2 = (int64_t)u.t2 * N + n;
    const float tab2 = (KIND == UPD_SAGAEM && u.t2 != u.t) ? u.table[q2] : tab;
    Neighbours nb;
    if (KIND != UPD_OSEM) nb = load_neighbours(u.f, ix, iy, p.nx, p.ny);
    // the stencil sums need only f and its neighbours: they run while the
    // first index/weight batch of the gather is in flight
    double D = 0.0, E = 0.0, gr = 0.0;
    const double b = bp_range_mid<U>(rowT, valT, beg, end, u.ratio, lig, [&] {
        if (p.beta > 0.0) {
            if (EM) surrogate_nb((double)f, nb, p, D, E);
            else if (KIND != UPD_OSEM) gr = penalty_grad_nb((double)f, nb, p);
        }
    });
    double b2 = b;
    if (KIND == UPD_SAGAEM && u.t2 != u.t) b2 = bp_group(ptrT, rowT, valT, q2, u.ratio2, lig);  // uniform branch
    if (lig != 0) return;
    float out;
    if (KIND == UPD_SAGAEM) {
        // Sec. 2.3, remark after eq. tempsvrem: the statistic uses the old entry
        // of subset t and the old table mean, then subset t2's entry is refreshed
        const float tau = tau_of(u.Ns, f, b);
        const double sh = (1.0 - u.alpha) * sh0 + u.alpha * (((double)tau - (double)tab) + Qn / (double)u.Ns);
        u.s_hat[n] = sh;
        const float tau2 = (u.t2 != u.t) ? tau_of(u.Ns, f, b2) : tau;
        u.Q[n] = Qn + ((double)tau2 - (double)tab2);
        u.table[q2] = tau2;
        const double bb = p.beta * D;
        const double cc = (p.beta * (double)f * D + p.beta * E) - sn;
        out = (float)mstep_root(sh, bb, cc, sn);
    } else if (KIND == UPD_OSEM) {
        out = osem_math(f, b, st);
    } else if (KIND == UPD_SVREM) {
        double sh;
        out = svrem_math(u.Ns, u.alpha, p.beta, f, b, sh0, tab, sanc, sn, D, E, &sh);
        u.s_hat[n] = sh;
    } else if (EM) {  // SEM
        const float tau = tau_of(u.Ns, f, b);
        const double sh = (1.0 - u.alpha) * sh0 + u.alpha * (double)tau;
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
    if (u.ft_out) u.ft_out[tiled_index_xy(ix, iy, u.tx)] = out;
}

// table entry (subset t, pixel n) from its back-projected sum b and f = f_n;
// the group's first lane writes it
template <int KIND>
__device__ inline void anchor_finish(const SnapArgs &a, int Ns, int64_t q, int n, float f, double b) {
    const PenaltyArgs &p = a.pen;
    double gr = 0.0;
    if (KIND != UPD_SVREM && KIND != UPD_SAGAEM && p.beta > 0.0) gr = a.grad ? a.grad[n] : penalty_grad_at(a.f, n, p);
    a.table[q] = (KIND == UPD_SVREM || KIND == UPD_SAGAEM) ? tau_of(Ns, f, b) : q_of(b, gr, p.beta, Ns);
}

template <int KIND, typename WT, typename IT>
__device__ inline void anchor_entry(const int *__restrict__ ptrT, const IT *__restrict__ rowT,
                                    const WT *__restrict__ valT, const int *__restrict__ row_start, int Ns, int N,
                                    const SnapArgs &a, int64_t q, int lig) {
    const int t = (int)(q / N), n = (int)(q - (int64_t)t * N);
    const PenaltyArgs &p = a.pen;
    constexpr bool GRAD = (KIND != UPD_SVREM && KIND != UPD_SAGAEM);  // q_t carries -(beta/Ns) grad R
    const float f = a.f[n];
    // the penalty gradient: the pixel's precomputed value, or (anchor_finish's,
    // from the same values) computed while the first index/weight batch of the
    // gather is in flight
    const bool own = GRAD && p.beta > 0.0 && !a.grad;
    double gr = (GRAD && p.beta > 0.0 && a.grad) ? a.grad[n] : 0.0;
    Neighbours nb;
    if (own) nb = load_neighbours_of(a.f, n, p);
    const double b = bp_range_mid(rowT, valT, ptrT[q], ptrT[q + 1], a.ratio_all + row_start[t], lig, [&] {
        if (own) gr = penalty_grad_nb((double)f, nb, p);
    });
    if (lig != 0) return;
    a.table[q] = GRAD ? q_of(b, gr, p.beta, Ns) : tau_of(Ns, f, b);
}

// Anchor sums of pixel n from the table: SVREM s_anc (and s_hat at a reset),
// SVRG g_tilde, SAGA / SAGA-EM Q (SAGA-EM also s_hat^0 = s(f^0)); returns the
// table sum over the subsets.  `mid()` runs while the first batch of table
// loads is in flight.
template <int KIND, class Mid>
__device__ inline double anchor_sum_pixel(const double *__restrict__ sens, int Ns, int N, const SnapArgs &a, int n,
                                         Mid mid) {
    const double sum = subset_sum_mid(a.table, Ns, N, n, mid);
    if (KIND == UPD_SVREM) {
        const double sa = sum / (double)Ns;
        a.s_anc[n] = sa;
        if (a.init_shat) a.s_hat[n] = sa;
    } else if (KIND == UPD_SVRG) {
        a.g_tilde[n] = (sum - sens[n]) / (double)Ns;
    } else if (KIND == UPD_SAGAEM) {  // table fill at k = 0: s_hat^0 = s(f^0)
        a.Q[n] = sum;
        a.s_hat[n] = sum / (double)Ns;
    } else {
        a.Q[n] = sum;
    }
    return sum;
}

template <int KIND>
__device__ inline double anchor_sum_pixel(const double *__restrict__ sens, int Ns, int N, const SnapArgs &a, int n) {
    return anchor_sum_pixel<KIND>(sens, Ns, N, a, n, [] {});
}

// The anchor sums of pixel n followed by the update of the iteration that
// takes the anchor.  There f = f_anc, so the subset term of subset u.t is the
// table entry itself (the same gather and the same expression computed it),
// and the update needs no forward projection or gather of its own:
//   SVREM: tau_t(f) - tau_anc_t = 0;  SVRG: q_t(f) - q_anc_t = 0;
//   SAGA (table fill at k = 0): q_t(f) - q_t = 0 and Q is unchanged;
//   SAGA-EM (table fill at k = 0): tau_t(f) - S_t = 0, and the refreshed
//   entry S_t2 = tau_t2(f) is already in the table (Q unchanged).
// `a` and `u` name the same state arrays (iterate, table, s_hat, s_anc, Q,
// g_tilde): the update takes the anchor quantities just computed instead of
// reading them back, and issues its own loads before the table sum.
template <int KIND>
__device__ inline void anchor_sum_update_pixel(const float *__restrict__ sens_t, const double *__restrict__ sens,
                                               int Ns, int N, const SnapArgs &a, const UpdateArgs &u, int n) {
    const int64_t q = (int64_t)u.t * N + n;
    const PenaltyArgs &p = u.pen;
    constexpr bool EM = (KIND == UPD_SVREM || KIND == UPD_SAGAEM);
    const float f = u.f[n];
    const float tab = u.table[q];
    const double sn = sens[n];
    const double sh_prev = (KIND == UPD_SVREM) ? u.s_hat[n] : 0.0;  // before a reset overwrites it
    const float st = !EM ? sens_t[q] : 0.0f;
    Neighbours nb;
    if (EM && p.beta > 0.0) nb = load_neighbours_of(u.f, n, p);
    double D = 0.0, E = 0.0;
    // the stencil sums run while the first batch of table loads is in flight
    const double sum = anchor_sum_pixel<KIND>(sens, Ns, N, a, n, [&] {
        if (EM && p.beta > 0.0) surrogate_nb((double)f, nb, p, D, E);
    });
    float out;
    if (KIND == UPD_SVREM) {
        const double sa = sum / (double)Ns;  // s_anc[n], and s_hat[n] at a reset
        double sh;
        out = svrem_math_tau(u.alpha, p.beta, f, tab, a.init_shat ? sa : sh_prev, tab, sa, sn, D, E, &sh);
        u.s_hat[n] = sh;
    } else if (KIND == UPD_SAGAEM) {
        const double sh =
            (1.0 - u.alpha) * (sum / (double)Ns) + u.alpha * (((double)tab - (double)tab) + sum / (double)u.Ns);
        u.s_hat[n] = sh;
        out = (float)mstep_root(sh, p.beta * D, (p.beta * (double)f * D + p.beta * E) - sn, sn);
    } else {
        double dir;
        if (KIND == UPD_SVRG) {
            dir = ((double)tab - (double)tab) + (sum - sn) / (double)Ns;  // g_tilde[n]
        } else {
            dir = ((double)tab - (double)tab) + (sum - sn) / (double)u.Ns;  // Q[n] = sum
            u.Q[n] = sum + ((double)tab - (double)tab);
        }
        const double d = precond_of(u, q, n, f, st);
        out = (float)fmax(0.0, (double)f + (u.alpha * d) * dir);
    }
    u.f_out[n] = out;
    if (u.ft_out) u.ft_out[tiled_index(n, p.nx, u.tx)] = out;
}

// frozen preconditioner entry i: d_t[n] = f0[n] / (A_t^T 1)[n] (per subset,
// i = t*N + n) or d[n] = f0[n] / (A^T 1)[n]; 0 where the sensitivity is 0
__device__ inline void precond_entry(const float *f0, const float *sens_t, const double *sens, int N,
                                     int per_subset, int64_t i, float *d) {
    if (per_subset) {
        const int n = (int)(i % N);
        const float st = sens_t[i];
        d[i] = st > 0.0f ? (float)((double)f0[n] / (double)st) : 0.0f;
    } else {
        d[i] = sens[i] > 0.0 ? (float)((double)f0[i] / sens[i]) : 0.0f;
    }
}

}  // namespace svr
