// Host side of the C ABI: argument validation, object lifetimes, and the
// epoch drivers that enqueue the projector and update kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "util.h"
#include "batch.h"
#include "trace.h"

using namespace svr;

struct svr_recon {
    Matrix *A = nullptr;
    svr_params p{};
    int S = 1;
    int device = 0;
    hipStream_t owner = nullptr;        // stream its memory was allocated on (freed there)
    int M = 0, N = 0, Ns = 0;
    float *g = nullptr, *w = nullptr;   // subset-ordered data
    float *f[2] = {nullptr, nullptr};   // ping-pong iterate
    float *ft = nullptr;                // the current iterate in tiled order (single slice; Nt floats)
    int cur = 0;
    float *ratio = nullptr;             // M, subset-ordered
    double *s_hat = nullptr, *s_anc = nullptr, *Q = nullptr, *g_tilde = nullptr;
    double *grad_anc = nullptr;         // SVRG / SAGA: grad R at the anchor, per pixel (N)
    float *table = nullptr;             // Ns*N
    float *dpre = nullptr;              // frozen preconditioner
    int dpre_per_subset = 0;
    double *part = nullptr;             // reduction partials
    int n_part = 0;
    double *scal = nullptr;             // 2 FP64 scalars
    int *bad = nullptr;                 // device flag / counter
    int64_t k = 0, n_snap = 0;
    bool numeric_error = false;
    // kernel timing: pairs of events bracketing launches, with their kind
    int *d_order = nullptr;             // device copy of an epoch's subset sequence
    int order_cap = 0;
    unsigned *d_sync = nullptr;         // grid barrier words of the persistent kernel
    int *d_status = nullptr;            // set by a persistent kernel that aborted
    int grid_cache[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    bool prof = false;
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_kind;
    size_t ev_used = 0;
    StackPlan plan;                     // slice stacks: image regions, row segments, schedules
};

namespace {
using Recon = svr_recon;

int kind_of_algo(int algo) {
    switch (algo) {
        case SVR_ALGO_OSEM: return UPD_OSEM;
        case SVR_ALGO_SVREM: return UPD_SVREM;
        case SVR_ALGO_SVRG: return UPD_SVRG;
        case SVR_ALGO_SAGA: return UPD_SAGA;
        case SVR_ALGO_SGA: return UPD_SGA;
        case SVR_ALGO_BSREM: return UPD_SGA;
        case SVR_ALGO_SEM: return UPD_SEM;
        case SVR_ALGO_SAGAEM: return UPD_SAGAEM;
    }
    return -1;
}

void free_recon(Recon *R) {
    if (!R) return;
    AllocStream as(R->owner);
    for (hipEvent_t e : R->ev) (void)hipEventDestroy(e);
    void *ptrs[] = {R->g, R->w, R->f[0], R->f[1], R->ft, R->ratio, R->s_hat, R->s_anc, R->Q, R->g_tilde, R->grad_anc,
                    R->table, R->dpre, R->part, R->scal, R->bad, R->d_order, R->d_sync, R->d_status};
    for (void *q : ptrs) dfree(q);
    ms_plan_free(R->plan);
    delete R;
}

// Arms the next kernel launch of this thread to carry a pair of timing events
// (start and end of the dispatch itself); no-op unless profiling.
int prof_begin(Recon *R, int kind, hipStream_t) {
    if (!R->prof) return SVR_OK;
    if (R->ev_used + 2 > R->ev.size()) {
        for (int i = 0; i < 2; ++i) {
            hipEvent_t e;
            SVR_HIP(hipEventCreate(&e));
            R->ev.push_back(e);
        }
        R->ev_kind.resize(R->ev.size() / 2);
    }
    R->ev_kind[R->ev_used / 2] = kind;
    LaunchEvents &t = pending_timing();
    t.start = R->ev[R->ev_used];
    t.stop = R->ev[R->ev_used + 1];
    return SVR_OK;
}
int prof_end(Recon *R, hipStream_t s) {
    if (!R->prof) return SVR_OK;
    LaunchEvents &t = pending_timing();
    if (t.start) {  // the armed launch did not happen (nothing to time)
        t.start = t.stop = nullptr;
        t.span = 1;
        return SVR_OK;
    }
    if (t.stop) {  // a span ended early: close it on the stream
        SVR_HIP(hipEventRecord(t.stop, s));
        t.stop = nullptr;
        t.span = 1;
    }
    R->ev_used += 2;
    return SVR_OK;
}

// eps of the modified likelihood (0 when it is off).  It enters the ratio of
// the gradient updates and the objective; the EM-type updates (the OSEM
// initialisation epochs of a gradient recon) keep the EM ratio.
double ll_eps_of(const Recon *R) { return (R->p.flags & SVR_FLAG_MODIFIED_LL) ? R->p.ll_eps : 0.0; }
double ll_eps_of(const Recon *R, int kind) {
    return (kind == UPD_SVRG || kind == UPD_SAGA || kind == UPD_SGA) ? ll_eps_of(R) : 0.0;
}

PenaltyArgs pen_of(const Recon *R) {
    return PenaltyArgs{R->p.penalty, R->p.delta, R->p.beta, R->A->geom.nx, R->A->geom.ny};
}

int check_geom(const svr_geometry *g) {
    SVR_REQUIRE(g, "geometry is NULL");
    SVR_REQUIRE(g->nx >= 1 && g->ny >= 1 && g->n_views >= 1 && g->n_bins >= 1, "sizes must be >= 1");
    SVR_REQUIRE((int64_t)g->nx * g->ny < (1ll << 30) && (int64_t)g->n_views * g->n_bins < (1ll << 30),
                "image or sinogram too large");
    SVR_REQUIRE(g->pixel_mm > 0 && g->bin_mm > 0 && std::isfinite(g->pixel_mm) && std::isfinite(g->bin_mm),
                "pixel_mm and bin_mm must be finite and > 0");
    SVR_REQUIRE(g->arc_rad > 0 && std::isfinite(g->arc_rad), "arc_rad must be finite and > 0");
    return SVR_OK;
}

int check_order(const Recon *R, const int32_t *order, int32_t n) {
    SVR_REQUIRE(n >= 0, "n must be >= 0");
    SVR_REQUIRE(n == 0 || order, "order is NULL");
    for (int i = 0; i < n; ++i)
        SVR_REQUIRE(order[i] >= 0 && order[i] < R->Ns, "order[%d] = %d outside [0, %d)", i, order[i], R->Ns);
    return SVR_OK;
}

// Anchor pass at the current image (ratio of all rows, then the table) fused
// with the update of the iteration that takes it (subset t): see
// anchor_sum_update_pixel.
int anchor_iteration(Recon *R, int kind, UpdateArgs &u, hipStream_t s) {
    TraceRange tr("svr.anchor");
    Matrix &A = *R->A;
    FwdArgs fa{R->ft, R->g, R->w, R->ratio, nullptr, nullptr};
    fa.eps = ll_eps_of(R, kind);
    int rc = prof_begin(R, 2, s);
    if (!rc) rc = launch_forward(A, 0, A.M, 1, fa, s);
    if (!rc) rc = prof_end(R, s);
    if (rc) return rc;
    SnapArgs sa{};
    sa.ratio_all = R->ratio;
    sa.f = R->f[R->cur];
    sa.table = R->table;
    sa.s_anc = R->s_anc;
    sa.s_hat = R->s_hat;
    sa.init_shat = (R->k == 0) || (R->p.flags & SVR_FLAG_RESET_SHAT_AT_ANCHOR);
    sa.g_tilde = R->g_tilde;
    sa.Q = R->Q;
    sa.pen = pen_of(R);
    if ((kind == UPD_SVRG || kind == UPD_SAGA) && sa.pen.beta > 0.0 && R->grad_anc) {
        // the table's penalty term, once per pixel instead of once per (subset, pixel)
        rc = launch_penalty_grad(A, sa.f, sa.pen, R->grad_anc, s);
        if (rc) return rc;
        sa.grad = R->grad_anc;
    }
    rc = prof_begin(R, 3, s);
    if (!rc) rc = launch_anchor_table(A, kind, sa, s);
    if (!rc) rc = prof_end(R, s);
    if (rc) return rc;
    if ((kind == UPD_SVRG || kind == UPD_SAGA) && R->k == 0 && R->p.precond != SVR_PRECOND_ITERATE) {
        rc = launch_precond(A, R->f[R->cur], R->dpre_per_subset, R->dpre, s);
        if (rc) return rc;
    }
    rc = prof_begin(R, 4, s);
    if (!rc) rc = launch_anchor_sum_update(A, kind, sa, u, s);
    if (!rc) rc = prof_end(R, s);
    if (rc) return rc;
    R->n_snap++;
    return SVR_OK;
}

// number of anchor (or table-fill) passes among iterations k0 .. k0+n-1
int64_t anchors_in(const Recon *R, int algo, int64_t k0, int n) {
    if (algo == SVR_ALGO_SVREM || algo == SVR_ALGO_SVRG) {
        const int64_t P = (int64_t)R->p.eta * R->Ns;
        return (k0 + n - 1) / P - (k0 - 1 >= 0 ? (k0 - 1) / P : -1);
    }
    if (algo == SVR_ALGO_SAGA || algo == SVR_ALGO_SAGAEM) return k0 == 0 ? 1 : 0;
    return 0;
}

// The update arguments of the iteration on subset t (SAGA-EM: refreshed
// subset t2) at the recon's current iterate and iteration count.
UpdateArgs iteration_args(const Recon *R, int algo, int t, int t2) {
    const Matrix &A = *R->A;
    UpdateArgs u{};
    u.t = t;
    u.Ns = R->Ns;
    u.ratio = R->ratio + A.row_start[t];
    u.f = R->f[R->cur];
    u.f_out = R->f[1 - R->cur];
    u.ft_out = R->ft;
    u.tx = A.tx;
    u.alpha = R->p.alpha;
    if (algo == SVR_ALGO_BSREM || algo == SVR_ALGO_SEM) u.alpha = R->p.alpha / (R->p.decay * (double)R->k + 1.0);
    u.s_hat = R->s_hat;
    u.s_anc = R->s_anc;
    u.table = R->table;
    u.Q = R->Q;
    u.g_tilde = R->g_tilde;
    u.dpre = (R->p.precond == SVR_PRECOND_ITERATE) ? nullptr : R->dpre;
    u.dpre_per_subset = R->dpre_per_subset;
    u.shat_zero = (algo == SVR_ALGO_SEM && R->k == 0);
    u.pen = pen_of(R);
    if (algo == SVR_ALGO_OSEM) u.pen.beta = 0.0;
    u.t2 = t2;
    u.ratio2 = R->ratio + A.row_start[t2];
    return u;
}

// whether the next iteration takes an anchor (SVREM, SVRG: every eta*Ns
// iterations) or fills the table (SAGA, SAGA-EM: the first)
bool is_anchor(const Recon *R, int algo) {
    return ((algo == SVR_ALGO_SVREM || algo == SVR_ALGO_SVRG) && R->k % ((int64_t)R->p.eta * R->Ns) == 0) ||
           ((algo == SVR_ALGO_SAGA || algo == SVR_ALGO_SAGAEM) && R->k == 0);
}

void advance_iteration(Recon *R, int algo) {
    R->cur = 1 - R->cur;
    if (algo != SVR_ALGO_OSEM) R->k++;
}

int run_epoch_persistent(Recon *R, int algo, int kind, const int32_t *order, int32_t n, hipStream_t s) {
    Matrix &A = *R->A;
    if (n > R->order_cap) {
        AllocStream as(s);
        dfree(R->d_order);  // stream-ordered after any earlier epoch reading it
        R->d_order = nullptr;
        R->order_cap = 0;
        SVR_HIP(dalloc(&R->d_order, n));
        R->order_cap = n;
    }
    // pageable source: the copy has consumed order[] when the call returns, and
    // it is stream-ordered after any earlier epoch still reading d_order
    SVR_HIP(hipMemcpyAsync(R->d_order, order, sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    SVR_HIP(hipMemsetAsync(R->d_sync, 0, sizeof(unsigned) * persistent_sync_words(), s));
    EpochArgs e{};
    e.row_ptr = A.d_row_ptr;
    e.col = A.d_colt;
    e.val = A.d_val;
    e.ptrT = A.d_ptrT;
    e.rowT = A.d_rowT;
    e.valT = A.d_valT;
    e.row_start = A.d_row_start;
    e.sens_t = A.d_sens_t;
    e.sens = A.d_sens;
    e.M = A.M;
    e.pair_rows = A.pair_rows_eff();
    e.N = A.N;
    e.Ns = A.Ns;
    e.g = R->g;
    e.w = R->w;
    e.ratio = R->ratio;
    e.f0 = R->f[0];
    e.f1 = R->f[1];
    e.cur0 = R->cur;
    e.ft = R->ft;
    e.tx = A.tx;
    e.eps = ll_eps_of(R, kind);
    e.s_hat = R->s_hat;
    e.s_anc = R->s_anc;
    e.Q = R->Q;
    e.g_tilde = R->g_tilde;
    e.table = R->table;
    e.dpre = (R->p.precond == SVR_PRECOND_ITERATE) ? nullptr : R->dpre;
    e.dpre_per_subset = R->dpre_per_subset;
    e.pen = pen_of(R);
    if (algo == SVR_ALGO_OSEM) e.pen.beta = 0.0;
    e.alpha = R->p.alpha;
    e.decay = R->p.decay;
    e.decaying = (algo == SVR_ALGO_BSREM || algo == SVR_ALGO_SEM);
    e.eta = R->p.eta;
    e.flags = R->p.flags;
    e.order = R->d_order;
    e.n = n;
    e.k0 = R->k;
    e.sync = R->d_sync;
    e.status = R->d_status;
    int rc = prof_begin(R, 5, s);
    if (!rc) rc = launch_epoch(A, kind, e, s, &R->grid_cache[kind]);
    if (!rc) rc = prof_end(R, s);
    if (rc) return rc;
    R->n_snap += anchors_in(R, algo, R->k, n);
    if (n & 1) R->cur = 1 - R->cur;
    if (algo != SVR_ALGO_OSEM) R->k += n;
    return SVR_OK;
}

// slice stacks: one sparse-times-dense product per phase (OSEM and SVREM)
int run_epoch_slices(Recon *R, int algo, int kind, const int32_t *order, int32_t n, hipStream_t s) {
    Matrix &A = *R->A;
    const int S = R->S;
    const int axial = (R->p.flags & SVR_FLAG_AXIAL_PENALTY) ? 1 : 0;
    if (kind != UPD_OSEM && kind != UPD_SVREM) {
        set_error("slice stacks (n_slices > 1) run OSEM and SVREM epochs");
        return SVR_EINVAL;
    }
    int rc = SVR_OK;
    for (int i = 0; i < n; ++i) {
        const int t = order[i];
        float *f = R->f[R->cur];
        if (kind == UPD_SVREM && R->k % ((int64_t)R->p.eta * R->Ns) == 0) {
            TraceRange tr("svr.anchor");
            rc = prof_begin(R, 2, s);
            if (!rc) rc = ms_forward(A, R->plan, -1, 1, S, f, R->g, R->w, R->ratio, nullptr, nullptr, s, nullptr);
            if (!rc) rc = prof_end(R, s);
            if (!rc) rc = prof_begin(R, 3, s);
            if (!rc) rc = ms_anchor_table(A, R->plan, S, R->ratio, f, R->table, s);
            if (!rc) rc = prof_end(R, s);
            if (!rc) rc = prof_begin(R, 4, s);
            if (!rc)
                rc = ms_anchor_sum(A, S, R->table, R->s_anc, R->s_hat,
                                   (R->k == 0) || (R->p.flags & SVR_FLAG_RESET_SHAT_AT_ANCHOR), s);
            if (!rc) rc = prof_end(R, s);
            if (rc) return rc;
            R->n_snap++;
        }
        const int r0 = A.row_start[t];
        rc = prof_begin(R, 0, s);
        if (!rc) rc = ms_forward(A, R->plan, t, 1, S, f, R->g, R->w, R->ratio, nullptr, nullptr, s, nullptr);
        if (!rc) rc = prof_end(R, s);
        if (rc) return rc;
        UpdateArgs u{};
        u.t = t;
        u.Ns = R->Ns;
        u.ratio = R->ratio + (int64_t)r0 * S;
        u.f = f;
        u.f_out = R->f[1 - R->cur];
        u.alpha = R->p.alpha;
        u.s_hat = R->s_hat;
        u.s_anc = R->s_anc;
        u.table = R->table;
        u.pen = pen_of(R);
        if (kind == UPD_OSEM) u.pen.beta = 0.0;
        rc = prof_begin(R, 1, s);
        if (!rc) rc = ms_update(A, R->plan, kind, S, axial, u, s);
        if (!rc) rc = prof_end(R, s);
        if (rc) return rc;
        R->cur = 1 - R->cur;
        if (algo != SVR_ALGO_OSEM) R->k++;
    }
    return SVR_OK;
}

// reports (once) a persistent kernel that left through its barrier time-out
int check_status(Recon *R, hipStream_t s) {
    int st = 0;
    SVR_HIP(hipMemcpyAsync(&st, R->d_status, sizeof(int), hipMemcpyDeviceToHost, s));
    SVR_HIP(hipStreamSynchronize(s));
    if (st) {
        (void)hipMemsetAsync(R->d_status, 0, sizeof(int), s);
        set_error("a persistent epoch kernel aborted at a grid barrier (time-out); results are invalid");
        return SVR_EDEVICE;
    }
    return SVR_OK;
}

int run_epoch(Recon *R, int algo, const int32_t *order, int32_t n, void *stream,
              const int32_t *refresh = nullptr) {
    TraceRange tr(epoch_range_name(algo));
    clear_error();
    SVR_REQUIRE(R, "recon is NULL");
    if (algo != SVR_ALGO_OSEM)
        SVR_REQUIRE(R->p.algo == algo, "recon was created for algo %d, epoch call is for algo %d", R->p.algo, algo);
    int rc = check_order(R, order, n);
    if (rc) return rc;
    if (refresh) {
        rc = check_order(R, refresh, n);
        if (rc) return rc;
    }
    SVR_HIP(hipSetDevice(R->device));
    hipStream_t s = (hipStream_t)stream;
    Matrix &A = *R->A;
    const int kind = kind_of_algo(algo);
    // OSEM is the initialiser: it leaves k at 0, so the next variance-reduced
    // call starts with a fresh anchor (or table fill) and frozen preconditioner
    if (algo == SVR_ALGO_OSEM) R->k = 0;
    if (R->S > 1) return run_epoch_slices(R, algo, kind, order, n, s);
    if (n > 0 && (R->p.flags & SVR_FLAG_PERSISTENT_EPOCH)) return run_epoch_persistent(R, algo, kind, order, n, s);
    for (int i = 0; i < n; ++i) {
        const int t = order[i];
        const int t2 = refresh ? refresh[i] : t;
        UpdateArgs u = iteration_args(R, algo, t, t2);
        if (is_anchor(R, algo)) {
            rc = anchor_iteration(R, kind, u, s);
            if (rc) return rc;
        } else {
            FwdArgs fa{R->ft, R->g, R->w, R->ratio, nullptr, nullptr};
            fa.eps = ll_eps_of(R, kind);
            rc = prof_begin(R, 0, s);
            if (!rc) rc = launch_forward(A, A.row_start[t], A.row_start[t + 1], 1, fa, s);
            if (!rc) rc = prof_end(R, s);
            if (!rc && algo == SVR_ALGO_SAGAEM && t2 != t) {  // the refreshed subset's statistic
                rc = prof_begin(R, 0, s);
                if (!rc) rc = launch_forward(A, A.row_start[t2], A.row_start[t2 + 1], 1, fa, s);
                if (!rc) rc = prof_end(R, s);
            }
            if (!rc) rc = prof_begin(R, 1, s);
            if (!rc) rc = launch_update(A, kind, u, s);
            if (!rc) rc = prof_end(R, s);
            if (rc) return rc;
        }
        advance_iteration(R, algo);
    }
    return SVR_OK;
}

}  // namespace

// ---- one iteration at a time (the batched server) ------------------------------
namespace svr {

int plan_iteration(svr_recon *R, int t, IterPlan *p) {
    SVR_REQUIRE(R && p, "NULL argument");
    SVR_REQUIRE(R->S == 1 && !(R->p.flags & SVR_FLAG_PERSISTENT_EPOCH) && R->p.algo != SVR_ALGO_SAGAEM,
                "iteration plans are for single-slice recons without the persistent flag or SAGA-EM");
    SVR_REQUIRE(t >= 0 && t < R->Ns, "subset %d outside [0, %d)", t, R->Ns);
    const Matrix &A = *R->A;
    const int algo = R->p.algo;
    p->A = &A;
    p->kind = kind_of_algo(algo);
    p->anchor = is_anchor(R, algo);
    p->r0 = A.row_start[t];
    p->r1 = A.row_start[t + 1];
    p->pair = forward_pairs_for(p->r1 - p->r0, A.pair_rows_eff());
    p->fa = FwdArgs{R->ft, R->g, R->w, R->ratio, nullptr, nullptr};
    p->fa.eps = ll_eps_of(R, p->kind);
    p->u = iteration_args(R, algo, t, t);
    return SVR_OK;
}

void end_iteration(svr_recon *R) { advance_iteration(R, R->p.algo); }

int plan_anchor(svr_recon *R, IterPlan &p, SnapArgs *sa) {
    SVR_REQUIRE(R && sa && p.anchor && p.kind == UPD_SVREM,
                "batched anchor passes are for SVREM iteration plans at an anchor");
    const Matrix &A = *R->A;
    // the arguments anchor_iteration gives its whole forward pass, table and sums
    p.fa = FwdArgs{R->ft, R->g, R->w, R->ratio, nullptr, nullptr};
    p.fa.eps = ll_eps_of(R, p.kind);
    p.r0 = 0;
    p.r1 = A.M;
    p.pair = forward_pairs_for(A.M, A.pair_rows_eff());
    *sa = SnapArgs{};
    sa->ratio_all = R->ratio;
    sa->f = R->f[R->cur];
    sa->table = R->table;
    sa->s_anc = R->s_anc;
    sa->s_hat = R->s_hat;
    sa->init_shat = (R->k == 0) || (R->p.flags & SVR_FLAG_RESET_SHAT_AT_ANCHOR);
    sa->g_tilde = R->g_tilde;
    sa->Q = R->Q;
    sa->pen = pen_of(R);
    R->n_snap++;
    return SVR_OK;
}

int objective_enqueue(svr_recon *R, hipStream_t s, ObjectiveHost *out) {
    const Matrix &A = *R->A;
    SVR_HIP(hipMemsetAsync(R->bad, 0, sizeof(int), s));
    int nb = 0, nbp = 0, rc;
    if (R->S == 1) {
        FwdArgs fa{R->ft, R->g, R->w, nullptr, R->part, R->bad};
        fa.eps = ll_eps_of(R);
        rc = launch_forward(A, 0, A.M, 2, fa, s, &nb);
    } else {
        rc = ms_forward(A, R->plan, -1, 2, R->S, R->f[R->cur], R->g, R->w, nullptr, R->part, R->bad, s, &nb);
    }
    if (!rc) rc = launch_reduce_sum(R->part, nb, R->scal, s);
    if (!rc) {
        if (R->S == 1)
            rc = launch_penalty_value(A, R->f[R->cur], R->p.penalty, R->p.delta, R->part, &nbp, s);
        else
            rc = ms_penalty_value(A, R->S, R->f[R->cur], R->p.penalty, R->p.delta,
                                  (R->p.flags & SVR_FLAG_AXIAL_PENALTY) ? 1 : 0, R->part, &nbp, s);
    }
    if (!rc) rc = launch_reduce_sum(R->part, nbp, R->scal + 1, s);
    if (rc) return rc;
    SVR_HIP(hipMemcpyAsync(out->sums, R->scal, sizeof(out->sums), hipMemcpyDeviceToHost, s));
    SVR_HIP(hipMemcpyAsync(&out->bad, R->bad, sizeof(int), hipMemcpyDeviceToHost, s));
    SVR_HIP(hipMemcpyAsync(&out->status, R->d_status, sizeof(int), hipMemcpyDeviceToHost, s));
    return SVR_OK;
}

int objective_result(svr_recon *R, const ObjectiveHost &o, hipStream_t s, double *phi_host) {
    if (o.status) {
        (void)hipMemsetAsync(R->d_status, 0, sizeof(int), s);
        set_error("a persistent epoch kernel aborted at a grid barrier (time-out); results are invalid");
        return SVR_EDEVICE;
    }
    const double phi = o.bad ? -INFINITY : o.sums[0] - R->p.beta * o.sums[1];
    *phi_host = phi;
    if (!std::isfinite(phi)) {
        R->numeric_error = true;
        set_error("objective is not finite (%g)", phi);
        return SVR_ENUMERIC;
    }
    return SVR_OK;
}

const float *current_image(const svr_recon *R) { return R->f[R->cur]; }

}  // namespace svr

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *svr_last_error(void) { return svr::last_error(); }
int svr_version(void) { return 10000; }

int svr_build_system_matrix(const svr_geometry *geom, int32_t n_subsets, int32_t wtype, const float *mu_dev,
                            void *stream, svr_matrix **out) {
    clear_error();
    TraceRange tr("svr.build_matrix");
    SVR_REQUIRE(out, "out is NULL");
    *out = nullptr;
    int rc = check_geom(geom);
    if (rc) return rc;
    SVR_REQUIRE(n_subsets >= 1 && n_subsets <= geom->n_views, "n_subsets must be in [1, n_views]");
    SVR_REQUIRE((int64_t)n_subsets * geom->nx * geom->ny < (1ll << 31), "n_subsets * nx * ny must be below 2^31");
    const int wbase = wtype & 0xff;
    SVR_REQUIRE((wtype & ~(0xff | SVR_W_INDEX32)) == 0 &&
                    (wbase == SVR_W_F32 || wbase == SVR_W_F16 || wbase == SVR_W_BF16),
                "unknown wtype %d", wtype);
    svr_matrix *A = new (std::nothrow) svr_matrix();
    SVR_REQUIRE(A, "host allocation failed");
    A->proj_mu = new (std::nothrow) std::mutex();
    if (!A->proj_mu) {
        delete A;
        set_error("host allocation failed");
        return SVR_ENOMEM;
    }
    A->geom = *geom;
    A->Ns = n_subsets;
    A->wtype = wbase;
    A->idx16 = (wtype & SVR_W_INDEX32) ? 0 : 1;
    (void)hipGetDevice(&A->device);
    if (hipDeviceGetAttribute(&A->cus, hipDeviceAttributeMultiprocessorCount, A->device) != hipSuccess || A->cus < 1)
        A->cus = 1;
    hipStream_t s = (hipStream_t)stream;
    if (mu_dev) {
        AllocStream as(s);
        int *cnt = nullptr;
        hipError_t e = dalloc(&cnt, 1);
        if (e != hipSuccess) { svr_matrix_destroy(A); set_error("allocation failed"); return SVR_ENOMEM; }
        (void)hipMemsetAsync(cnt, 0, sizeof(int), s);
        launch_count_bad(mu_dev, (int64_t)geom->nx * geom->ny, 0, cnt, s);
        int h = 0;
        (void)hipMemcpyAsync(&h, cnt, sizeof(int), hipMemcpyDeviceToHost, s);
        (void)hipStreamSynchronize(s);
        dfree(cnt);
        if (h) { svr_matrix_destroy(A); set_error("mu has %d negative or non-finite entries", h); return SVR_EINVAL; }
    }
    rc = build_matrix(*A, mu_dev, s);
    if (rc) {
        svr_matrix_destroy(A);
        return rc;
    }
    *out = A;
    return SVR_OK;
}

int svr_matrix_info(const svr_matrix *A, svr_matrix_info_t *info, int64_t *nnz_per_subset) {
    clear_error();
    SVR_REQUIRE(A && info, "NULL argument");
    info->nnz = A->nnz;
    info->bytes = A->bytes;
    info->n_subsets = A->Ns;
    info->n_rows = A->M;
    info->n_pixels = A->N;
    info->max_row_nnz = A->max_row_nnz;
    info->max_col_nnz = A->max_col_nnz;
    info->wtype = A->wtype;
    info->index_bytes = A->ibytes();
    if (nnz_per_subset)
        for (int t = 0; t < A->Ns; ++t) nnz_per_subset[t] = A->nnz_sub[t];
    return SVR_OK;
}

static float host_w(const void *base, int wtype, int64_t i) {
    if (wtype == SVR_W_F32) return ((const float *)base)[i];
    if (wtype == SVR_W_F16) return (float)((const _Float16 *)base)[i];
    uint32_t u = (uint32_t)((const uint16_t *)base)[i] << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

int svr_matrix_export(const svr_matrix *A, int32_t which, int32_t *ptr, int32_t *idx, float *val) {
    clear_error();
    SVR_REQUIRE(A, "matrix is NULL");
    SVR_REQUIRE(which == 0 || which == 1, "which must be 0 or 1");
    SVR_HIP(hipSetDevice(A->device));
    const int64_t nnz = A->nnz;
    const int wb = A->wbytes();
    const int ib = A->ibytes();
    auto idx_host = [&](const void *dev, std::vector<int> &out) -> int {
        out.resize(nnz);
        if (ib == 4) {
            SVR_HIP(hipMemcpy(out.data(), dev, sizeof(int) * nnz, hipMemcpyDeviceToHost));
        } else {
            std::vector<uint16_t> t(nnz);
            SVR_HIP(hipMemcpy(t.data(), dev, sizeof(uint16_t) * nnz, hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < nnz; ++i) out[i] = t[i];
        }
        return SVR_OK;
    };
    if (which == 0) {
        std::vector<int> rp(A->M + 1), rs(A->M), col;
        std::vector<char> v(nnz * wb);
        SVR_HIP(hipMemcpy(rp.data(), A->d_row_ptr, sizeof(int) * (A->M + 1), hipMemcpyDeviceToHost));
        SVR_HIP(hipMemcpy(rs.data(), A->d_row_sino, sizeof(int) * A->M, hipMemcpyDeviceToHost));
        int rc = idx_host(A->d_col, col);
        if (rc) return rc;
        SVR_HIP(hipMemcpy(v.data(), A->d_val, (size_t)wb * nnz, hipMemcpyDeviceToHost));
        std::vector<int> inv(A->M);
        for (int r = 0; r < A->M; ++r) inv[rs[r]] = r;
        int64_t pos = 0;
        if (ptr) ptr[0] = 0;
        for (int m = 0; m < A->M; ++m) {
            const int r = inv[m];
            for (int i = rp[r]; i < rp[r + 1]; ++i, ++pos) {
                if (idx) idx[pos] = col[i];
                if (val) val[pos] = host_w(v.data(), A->wtype, i);
            }
            if (ptr) ptr[m + 1] = (int32_t)pos;
        }
    } else {
        const int64_t NT = (int64_t)A->Ns * A->N;
        if (ptr) SVR_HIP(hipMemcpy(ptr, A->d_ptrT, sizeof(int) * (NT + 1), hipMemcpyDeviceToHost));
        if (idx) {
            std::vector<int> r;
            int rc = idx_host(A->d_rowT, r);
            if (rc) return rc;
            memcpy(idx, r.data(), sizeof(int) * nnz);
        }
        if (val) {
            std::vector<char> v(nnz * wb);
            SVR_HIP(hipMemcpy(v.data(), A->d_valT, (size_t)wb * nnz, hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < nnz; ++i) val[i] = host_w(v.data(), A->wtype, i);
        }
    }
    return SVR_OK;
}

__global__ static void k_f32_to_f64(const float *x, int n, double *y) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (double)x[i];
}

int svr_sensitivity(const svr_matrix *A, int32_t subset, double *out_dev, void *stream) {
    clear_error();
    SVR_REQUIRE(A && out_dev, "NULL argument");
    SVR_REQUIRE(subset >= -1 && subset < A->Ns, "subset %d out of range", subset);
    SVR_HIP(hipSetDevice(A->device));
    hipStream_t s = (hipStream_t)stream;
    if (subset < 0) {
        SVR_HIP(hipMemcpyAsync(out_dev, A->d_sens, sizeof(double) * A->N, hipMemcpyDeviceToDevice, s));
    } else {
        k_f32_to_f64<<<(A->N + 255) / 256, 256, 0, s>>>(A->d_sens_t + (int64_t)subset * A->N, A->N, out_dev);
        SVR_HIP(hipGetLastError());
    }
    return SVR_OK;
}

void svr_matrix_destroy(svr_matrix *A) {
    if (!A) return;
    TraceRange tr("svr.matrix_destroy");
    (void)hipSetDevice(A->device);
    if (A->proj_scratch) {  // the last projector call that used it has finished with it
        (void)hipEventSynchronize(A->proj_done);
        (void)hipFree(A->proj_scratch);
        (void)hipEventDestroy(A->proj_done);
    }
    delete A->proj_mu;
    AllocStream as(A->owner);
    void *ptrs[] = {A->d_row_start, A->d_row_sino, A->d_row_ptr, A->d_col, A->d_colt, A->d_val, A->d_ptrT,
                    A->d_rowT, A->d_valT, A->d_sens_t, A->d_sens};
    for (void *q : ptrs) dfree(q);
    delete A;
}

}  // extern "C"

namespace {

// n floats of scratch for a projector call on stream s: the matrix's kept buffer when it is idle
// and its last use was on s (stream order) or has completed, else a stream-ordered allocation of
// the call's own (*own = true).  Returns null when no memory could be had.
float *acquire_proj_scratch(const Matrix &A, size_t n, hipStream_t s, bool *own) {
    *own = false;
    {
        std::lock_guard<std::mutex> lk(*A.proj_mu);
        const size_t cap = std::max<size_t>((size_t)A.Nt, (size_t)A.M);
        if (!A.proj_busy && n <= cap) {
            if (!A.proj_scratch) {
                float *p = nullptr;
                hipEvent_t e = nullptr;
                if (hipMalloc((void **)&p, sizeof(float) * cap) == hipSuccess &&
                    hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess) {
                    A.proj_scratch = p;
                    A.proj_done = e;
                    A.proj_stream = s;  // no earlier use to wait for
                } else {
                    if (p) (void)hipFree(p);
                    (void)hipGetLastError();
                }
            }
            if (A.proj_scratch && (A.proj_stream == s || hipEventQuery(A.proj_done) == hipSuccess)) {
                A.proj_busy = true;
                return A.proj_scratch;
            }
            (void)hipGetLastError();  // hipEventQuery's "not ready"
        }
    }
    *own = true;
    float *p = nullptr;
    if (hipMallocAsync((void **)&p, sizeof(float) * n, s) != hipSuccess) return nullptr;
    return p;
}

void release_proj_scratch(const Matrix &A, float *p, bool own, hipStream_t s) {
    if (!p) return;
    if (own) {
        (void)hipFreeAsync(p, s);
        return;
    }
    std::lock_guard<std::mutex> lk(*A.proj_mu);
    (void)hipEventRecord(A.proj_done, s);
    A.proj_stream = s;
    A.proj_busy = false;
}

}  // namespace

extern "C" {

int svr_project(const svr_matrix *A, int32_t subset, const float *x_dev, int32_t n_slices, float *y_dev,
                void *stream) {
    clear_error();
    TraceRange tr("svr.project");
    SVR_REQUIRE(A && x_dev && y_dev, "NULL argument");
    SVR_REQUIRE(subset >= -1 && subset < A->Ns, "subset %d out of range", subset);
    SVR_REQUIRE(n_slices >= 1, "n_slices must be >= 1");
    SVR_HIP(hipSetDevice(A->device));
    hipStream_t s = (hipStream_t)stream;
    const int r0 = subset < 0 ? 0 : A->row_start[subset];
    const int r1 = subset < 0 ? A->M : A->row_start[subset + 1];
    bool own = false;
    float *xt = acquire_proj_scratch(*A, (size_t)A->Nt, s, &own);  // each slice in the tiled order
    SVR_REQUIRE(xt, "no device memory for the projector's scratch");
    int rc = SVR_OK;
    for (int sl = 0; sl < n_slices && rc == SVR_OK; ++sl) {
        rc = launch_tile_image(*A, x_dev + (int64_t)sl * A->N, xt, s);
        FwdArgs fa{xt, nullptr, nullptr, y_dev + (int64_t)sl * A->M, nullptr, nullptr};
        if (rc == SVR_OK) rc = launch_forward(*A, r0, r1, 0, fa, s);
    }
    release_proj_scratch(*A, xt, own, s);
    return rc;
}

}  // extern "C"

// Scratch of svr_project_noalloc: the tiled copy of one slice of the image.
// The library never allocates it; each device holds its own copy for the life
// of the process.  Host code must not pass `scratch` itself to a kernel (it is
// a host-side stand-in): it uses the device address looked up per device.
static __device__ __align__(256) float scratch[SVR_NOALLOC_SCRATCH_FLOATS];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_dev[kMaxScratchDevices];  // device address of `scratch`, per device

// The address of `scratch` on `device` (the current device), looked up on the
// first call there with hipGetSymbolAddress and kept.
int noalloc_scratch(int device, float **out) {
    SVR_REQUIRE(device >= 0 && device < kMaxScratchDevices, "device %d beyond the %d supported", device,
                kMaxScratchDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *p = nullptr;
        SVR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        SVR_REQUIRE(p, "no device address for the scratch array");
        g_scratch_dev[device] = (float *)p;
    }
    *out = g_scratch_dev[device];
    return SVR_OK;
}

}  // namespace

extern "C" {

int svr_project_noalloc(const svr_matrix *A, int32_t subset, const float *x_dev, int32_t n_slices, float *y_dev,
                        void *stream) {
    clear_error();
    TraceRange tr("svr.project_noalloc");
    SVR_REQUIRE(A && x_dev && y_dev, "NULL argument");
    SVR_REQUIRE(subset >= -1 && subset < A->Ns, "subset %d out of range", subset);
    SVR_REQUIRE(n_slices >= 1, "n_slices must be >= 1");
    SVR_REQUIRE((int64_t)A->Nt <= (int64_t)SVR_NOALLOC_SCRATCH_FLOATS,
                "the tiled image (%d floats) exceeds the allocation-free scratch (%d floats)", A->Nt,
                (int)SVR_NOALLOC_SCRATCH_FLOATS);
    SVR_HIP(hipSetDevice(A->device));
    float *xt = nullptr;
    int rc = noalloc_scratch(A->device, &xt);
    if (rc != SVR_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int r0 = subset < 0 ? 0 : A->row_start[subset];
    const int r1 = subset < 0 ? A->M : A->row_start[subset + 1];
    for (int sl = 0; sl < n_slices && rc == SVR_OK; ++sl) {  // the same kernels as svr_project
        rc = launch_tile_image(*A, x_dev + (int64_t)sl * A->N, xt, s);
        FwdArgs fa{xt, nullptr, nullptr, y_dev + (int64_t)sl * A->M, nullptr, nullptr};
        if (rc == SVR_OK) rc = launch_forward(*A, r0, r1, 0, fa, s);
    }
    return rc;
}

int svr_backproject(const svr_matrix *A, int32_t subset, const float *y_dev, int32_t n_slices, float *x_dev,
                    void *stream) {
    clear_error();
    TraceRange tr("svr.backproject");
    SVR_REQUIRE(A && x_dev && y_dev, "NULL argument");
    SVR_REQUIRE(subset >= -1 && subset < A->Ns, "subset %d out of range", subset);
    SVR_REQUIRE(n_slices >= 1, "n_slices must be >= 1");
    SVR_HIP(hipSetDevice(A->device));
    hipStream_t s = (hipStream_t)stream;
    bool own = false;
    float *ysub = acquire_proj_scratch(*A, (size_t)A->M, s, &own);  // each slice in subset order
    SVR_REQUIRE(ysub, "no device memory for the projector's scratch");
    int rc = SVR_OK;
    for (int sl = 0; sl < n_slices && rc == SVR_OK; ++sl) {
        rc = launch_gather_rows(*A, y_dev + (int64_t)sl * A->M, ysub, s);
        if (rc == SVR_OK) rc = launch_backproject(*A, subset, ysub, x_dev + (int64_t)sl * A->N, s);
    }
    release_proj_scratch(*A, ysub, own, s);
    return rc;
}

int svr_recon_create(svr_matrix *A, const float *g_dev, const float *w_dev, const float *f0_dev, int32_t n_slices,
                     const svr_params *p, void *stream, svr_recon **out) {
    clear_error();
    TraceRange tr("svr.recon_create");
    SVR_REQUIRE(out, "out is NULL");
    *out = nullptr;
    SVR_REQUIRE(A && g_dev && w_dev && f0_dev && p, "NULL argument");
    SVR_REQUIRE(n_slices >= 1, "n_slices must be >= 1");
    SVR_REQUIRE(n_slices == 1 || p->algo == SVR_ALGO_SVREM || p->algo == SVR_ALGO_OSEM,
                "slice stacks (n_slices > 1) run OSEM and SVREM");
    // the stack kernels address an image or sinogram block with 32-bit byte
    // offsets (buffer loads)
    SVR_REQUIRE(n_slices == 1 || ((int64_t)A->N * n_slices * 4 <= INT32_MAX && (int64_t)A->M * n_slices * 4 <= INT32_MAX),
                "slice stack too large: %d slices x %d pixels / %d rows exceeds 2^31 bytes per block", n_slices, A->N,
                A->M);
    SVR_REQUIRE(kind_of_algo(p->algo) >= 0, "unknown algo %d", p->algo);
    SVR_REQUIRE(p->alpha > 0 && std::isfinite(p->alpha), "alpha must be finite and > 0");
    SVR_REQUIRE(p->beta >= 0 && std::isfinite(p->beta), "beta must be finite and >= 0");
    SVR_REQUIRE(p->eta >= 1, "eta must be >= 1");
    SVR_REQUIRE(p->penalty >= SVR_PEN_QUADRATIC && p->penalty <= SVR_PEN_HYPERBOLA, "unknown penalty %d",
                p->penalty);
    SVR_REQUIRE(p->penalty == SVR_PEN_QUADRATIC || (p->delta > 0 && std::isfinite(p->delta)),
                "delta must be finite and > 0");
    SVR_REQUIRE(p->precond >= 0 && p->precond <= 2, "unknown precond %d", p->precond);
    SVR_REQUIRE(p->decay >= 0 && std::isfinite(p->decay), "decay must be finite and >= 0");
    SVR_REQUIRE((p->flags & ~(SVR_FLAG_RESET_SHAT_AT_ANCHOR | SVR_FLAG_AXIAL_PENALTY | SVR_FLAG_PERSISTENT_EPOCH |
                              SVR_FLAG_MODIFIED_LL)) == 0,
                "unknown flags 0x%x", p->flags);
    if (p->flags & SVR_FLAG_MODIFIED_LL) {
        SVR_REQUIRE(p->algo == SVR_ALGO_SVRG || p->algo == SVR_ALGO_SAGA || p->algo == SVR_ALGO_SGA ||
                        p->algo == SVR_ALGO_BSREM,
                    "the modified likelihood (Sec. 2.3) is for the gradient algos SVRG, SAGA, SGA and BSREM");
        SVR_REQUIRE(p->ll_eps > 0 && std::isfinite(p->ll_eps), "ll_eps must be finite and > 0");
    }
    SVR_REQUIRE(!(p->flags & SVR_FLAG_PERSISTENT_EPOCH) || p->algo != SVR_ALGO_SAGAEM,
                "the persistent epoch kernel does not run SAGAEM");
    SVR_HIP(hipSetDevice(A->device));
    hipStream_t s = (hipStream_t)stream;
    svr_recon *R = new (std::nothrow) svr_recon();
    SVR_REQUIRE(R, "host allocation failed");
    AllocStream as(s);
    R->owner = s;
    R->A = A;
    R->p = *p;
    R->S = n_slices;
    R->device = A->device;
    R->M = A->M;
    R->N = A->N;
    R->Ns = A->Ns;
    const int M = A->M, N = A->N, Ns = A->Ns;
    const int64_t S = n_slices;
    const int64_t NT = (int64_t)Ns * N * S;
    const int64_t MS_ = (int64_t)M * S, NS_ = (int64_t)N * S;
    const int64_t nch = (S + 63) / 64;
    R->n_part = (int)std::max<int64_t>(std::max<int64_t>((M * nch + 3) / 4, (NS_ + 255) / 256), M) + 1;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (x != hipSuccess && e == hipSuccess) e = x; };
    chk(dalloc(&R->g, MS_));
    chk(dalloc(&R->w, MS_));
    chk(dalloc(&R->f[0], NS_));
    chk(dalloc(&R->f[1], NS_));
    if (S == 1) chk(dalloc(&R->ft, A->Nt));
    chk(dalloc(&R->ratio, MS_));
    chk(dalloc(&R->part, R->n_part));
    chk(dalloc(&R->scal, 2));
    chk(dalloc(&R->bad, 1));
    chk(dalloc(&R->d_sync, persistent_sync_words()));
    chk(dalloc(&R->d_status, 1));
    const int algo = p->algo;
    if (algo == SVR_ALGO_SVREM || algo == SVR_ALGO_SEM || algo == SVR_ALGO_SAGAEM) chk(dalloc(&R->s_hat, NS_));
    if (algo == SVR_ALGO_SVREM) chk(dalloc(&R->s_anc, NS_));
    if (algo == SVR_ALGO_SVREM || algo == SVR_ALGO_SVRG || algo == SVR_ALGO_SAGA || algo == SVR_ALGO_SAGAEM)
        chk(dalloc(&R->table, NT));
    if (algo == SVR_ALGO_SVRG) chk(dalloc(&R->g_tilde, N));
    if (algo == SVR_ALGO_SVRG || algo == SVR_ALGO_SAGA) chk(dalloc(&R->grad_anc, N));
    if (algo == SVR_ALGO_SAGA || algo == SVR_ALGO_SAGAEM) chk(dalloc(&R->Q, N));
    if ((algo == SVR_ALGO_SVRG || algo == SVR_ALGO_SAGA) && p->precond != SVR_PRECOND_ITERATE) {
        R->dpre_per_subset = (p->precond == SVR_PRECOND_SUBSET_FROZEN);
        chk(dalloc(&R->dpre, R->dpre_per_subset ? NT : (int64_t)N));
    }
    if (e != hipSuccess) {
        free_recon(R);
        set_error("device allocation failed: %s", hipGetErrorString(e));
        return SVR_ENOMEM;
    }
    // validate the data on the device
    SVR_HIP(hipMemsetAsync(R->bad, 0, sizeof(int), s));
    int rc = launch_count_bad(g_dev, MS_, 0, R->bad, s);
    if (!rc) rc = launch_count_bad(w_dev, MS_, 0, R->bad, s);
    int nbad_gw = 0, nbad_f = 0;
    if (!rc) {
        SVR_HIP(hipMemcpyAsync(&nbad_gw, R->bad, sizeof(int), hipMemcpyDeviceToHost, s));
        SVR_HIP(hipMemsetAsync(R->bad, 0, sizeof(int), s));
        rc = launch_count_bad(f0_dev, NS_, 1, R->bad, s);
    }
    if (!rc) {
        SVR_HIP(hipMemcpyAsync(&nbad_f, R->bad, sizeof(int), hipMemcpyDeviceToHost, s));
        SVR_HIP(hipStreamSynchronize(s));
    }
    if (rc || nbad_gw || nbad_f) {
        free_recon(R);
        if (!rc) {
            set_error("invalid data: %d negative/non-finite entries in g or w, %d non-positive/non-finite in f0",
                      nbad_gw, nbad_f);
            rc = SVR_EINVAL;
        }
        return rc;
    }
    if (S == 1) {
        rc = launch_gather_rows(*A, g_dev, R->g, s);
        if (!rc) rc = launch_gather_rows(*A, w_dev, R->w, s);
        if (!rc && hipMemcpyAsync(R->f[0], f0_dev, sizeof(float) * N, hipMemcpyDeviceToDevice, s) != hipSuccess)
            rc = SVR_EDEVICE;
        if (!rc) rc = launch_tile_image(*A, R->f[0], R->ft, s);
    } else {
        rc = ms_pack_sino(*A, (int)S, g_dev, R->g, s);
        if (!rc) rc = ms_pack_sino(*A, (int)S, w_dev, R->w, s);
        if (!rc) rc = ms_pack_img(N, (int)S, f0_dev, R->f[0], s);
        if (!rc) rc = ms_plan_build(*A, (int)S, R->plan, s);
    }
    if (rc) { free_recon(R); return rc; }
    SVR_HIP(hipMemsetAsync(R->ratio, 0, sizeof(float) * MS_, s));
    SVR_HIP(hipMemsetAsync(R->d_status, 0, sizeof(int), s));
    if (R->s_hat) SVR_HIP(hipMemsetAsync(R->s_hat, 0, sizeof(double) * NS_, s));
    SVR_HIP(hipStreamSynchronize(s));
    *out = R;
    return SVR_OK;
}

int svr_osem_epoch(svr_recon *R, const int32_t *o, int32_t n, void *s) { return run_epoch(R, SVR_ALGO_OSEM, o, n, s); }
int svr_svrem_epoch(svr_recon *R, const int32_t *o, int32_t n, void *s) { return run_epoch(R, SVR_ALGO_SVREM, o, n, s); }
int svr_svrg_epoch(svr_recon *R, const int32_t *o, int32_t n, void *s) { return run_epoch(R, SVR_ALGO_SVRG, o, n, s); }
int svr_saga_epoch(svr_recon *R, const int32_t *o, int32_t n, void *s) { return run_epoch(R, SVR_ALGO_SAGA, o, n, s); }
int svr_sga_epoch(svr_recon *R, const int32_t *o, int32_t n, void *s) { return run_epoch(R, SVR_ALGO_SGA, o, n, s); }
int svr_bsrem_epoch(svr_recon *R, const int32_t *o, int32_t n, void *s) { return run_epoch(R, SVR_ALGO_BSREM, o, n, s); }
int svr_sem_epoch(svr_recon *R, const int32_t *o, int32_t n, void *s) { return run_epoch(R, SVR_ALGO_SEM, o, n, s); }
int svr_sagaem_epoch(svr_recon *R, const int32_t *o, const int32_t *refresh, int32_t n, void *s) {
    return run_epoch(R, SVR_ALGO_SAGAEM, o, n, s, refresh);
}

int svr_objective(svr_recon *R, double *phi_host, void *stream) {
    clear_error();
    TraceRange tr("svr.objective");
    SVR_REQUIRE(R && phi_host, "NULL argument");
    SVR_HIP(hipSetDevice(R->device));
    hipStream_t s = (hipStream_t)stream;
    svr::ObjectiveHost o{};
    const int rc = svr::objective_enqueue(R, s, &o);
    if (rc) return rc;
    SVR_HIP(hipStreamSynchronize(s));
    return svr::objective_result(R, o, s, phi_host);
}

int svr_get_image(const svr_recon *R, float *f_dev, void *stream) {
    clear_error();
    SVR_REQUIRE(R && f_dev, "NULL argument");
    SVR_HIP(hipSetDevice(R->device));
    if (R->S == 1) {
        SVR_HIP(hipMemcpyAsync(f_dev, R->f[R->cur], sizeof(float) * R->N, hipMemcpyDeviceToDevice,
                               (hipStream_t)stream));
        return SVR_OK;
    }
    return ms_unpack_img(R->N, R->S, R->f[R->cur], f_dev, (hipStream_t)stream);
}

}  // extern "C"

// ---- state (checkpoint / resume) ---------------------------------------------
namespace {
struct Field {
    void *dev;
    size_t bytes;
};
std::vector<Field> state_fields(const Recon *R) {
    const size_t N = (size_t)R->N * R->S, NT = (size_t)R->Ns * R->N * R->S;
    std::vector<Field> v;
    v.push_back({R->f[R->cur], 4 * N});
    if (R->s_hat) v.push_back({R->s_hat, 8 * N});
    if (R->s_anc) v.push_back({R->s_anc, 8 * N});
    if (R->Q) v.push_back({R->Q, 8 * N});
    if (R->g_tilde) v.push_back({R->g_tilde, 8 * N});
    if (R->table) v.push_back({R->table, 4 * NT});
    if (R->dpre) v.push_back({R->dpre, 4 * (R->dpre_per_subset ? (size_t)R->Ns * R->N : (size_t)R->N)});
    return v;
}
struct StateHeader {
    uint64_t magic;
    int64_t k, n_snap;
    int32_t algo, Ns, N, M;
};
constexpr uint64_t STATE_MAGIC = 0x5356524553544154ull;
}  // namespace

extern "C" {

int svr_recon_info(const svr_recon *R, svr_recon_info_t *info) {
    clear_error();
    SVR_REQUIRE(R && info, "NULL argument");
    info->k = R->k;
    info->n_snapshots = R->n_snap;
    info->n_subsets = R->Ns;
    info->n_slices = R->S;
    info->n_pixels = R->N;
    info->n_rows = R->M;
    size_t tot = sizeof(StateHeader);
    for (auto &f : state_fields(R)) tot += f.bytes;
    info->state_bytes = (int64_t)tot;
    return SVR_OK;
}

int svr_recon_get_state(const svr_recon *R, void *buf, size_t *len, void *stream) {
    clear_error();
    TraceRange tr("svr.get_state");
    SVR_REQUIRE(R && len, "NULL argument");
    auto fields = state_fields(R);
    size_t tot = sizeof(StateHeader);
    for (auto &f : fields) tot += f.bytes;
    if (!buf) { *len = tot; return SVR_OK; }
    SVR_REQUIRE(*len >= tot, "buffer too small (%zu < %zu)", *len, tot);
    SVR_HIP(hipSetDevice(R->device));
    hipStream_t s = (hipStream_t)stream;
    int rc = check_status(const_cast<Recon *>(R), s);
    if (rc) return rc;
    StateHeader h{STATE_MAGIC, R->k, R->n_snap, R->p.algo, R->Ns, R->N, R->M};
    memcpy(buf, &h, sizeof(h));
    char *p = (char *)buf + sizeof(h);
    for (auto &f : fields) {
        SVR_HIP(hipMemcpyAsync(p, f.dev, f.bytes, hipMemcpyDeviceToHost, s));
        p += f.bytes;
    }
    SVR_HIP(hipStreamSynchronize(s));
    *len = tot;
    return SVR_OK;
}

int svr_recon_set_state(svr_recon *R, const void *buf, size_t len, void *stream) {
    clear_error();
    TraceRange tr("svr.set_state");
    SVR_REQUIRE(R && buf, "NULL argument");
    SVR_REQUIRE(len >= sizeof(StateHeader), "buffer too small");
    StateHeader h;
    memcpy(&h, buf, sizeof(h));
    SVR_REQUIRE(h.magic == STATE_MAGIC, "not a recon state");
    SVR_REQUIRE(h.algo == R->p.algo && h.Ns == R->Ns && h.N == R->N && h.M == R->M,
                "state was saved from a different problem or algorithm");
    SVR_HIP(hipSetDevice(R->device));
    hipStream_t s = (hipStream_t)stream;
    auto fields = state_fields(R);
    size_t tot = sizeof(StateHeader);
    for (auto &f : fields) tot += f.bytes;
    SVR_REQUIRE(len == tot, "state size %zu does not match %zu", len, tot);
    const char *p = (const char *)buf + sizeof(h);
    for (auto &f : fields) {
        SVR_HIP(hipMemcpyAsync(f.dev, p, f.bytes, hipMemcpyHostToDevice, s));
        p += f.bytes;
    }
    if (R->ft) {
        int rc = launch_tile_image(*R->A, R->f[R->cur], R->ft, s);
        if (rc) return rc;
    }
    SVR_HIP(hipStreamSynchronize(s));
    R->k = h.k;
    R->n_snap = h.n_snap;
    return SVR_OK;
}

int svr_recon_set_profiling(svr_recon *R, int32_t enable) {
    clear_error();
    SVR_REQUIRE(R, "recon is NULL");
    R->prof = enable != 0;
    return SVR_OK;
}

int svr_recon_kernel_times(svr_recon *R, svr_kernel_times_t *out) {
    clear_error();
    SVR_REQUIRE(R && out, "NULL argument");
    SVR_HIP(hipSetDevice(R->device));
    memset(out, 0, sizeof(*out));
    for (size_t i = 0; i < R->ev_used; i += 2) {
        SVR_HIP(hipEventSynchronize(R->ev[i + 1]));
        float ms = 0.0f;
        SVR_HIP(hipEventElapsedTime(&ms, R->ev[i], R->ev[i + 1]));
        const int k = R->ev_kind[i / 2];
        out->launches[k] += 1;
        out->total_ms[k] += ms;
    }
    R->ev_used = 0;
    return SVR_OK;
}

void svr_recon_destroy(svr_recon *R) {
    if (!R) return;
    TraceRange tr("svr.recon_destroy");
    (void)hipSetDevice(R->device);
    free_recon(R);
}

}  // extern "C"
