// Batched subset iterations for the server: one launch per phase runs the
// current iteration of several independent reconstructions.  Work items are
// (request, row block) for the forward and (request, pixel block) for the
// update; each item calls the single-request device functions with that
// request's own arguments, so every request's result is bitwise the one of
// its own epoch calls.
#pragma once

#include "common.h"

struct svr_recon;

namespace svr {

// The next iteration of a single-slice recon on subset t: either an anchor
// (or table fill; plan_anchor below prepares an SVREM one for the batched
// launches), or the arguments of the subset forward and update.
// end_iteration advances the recon after either.
struct IterPlan {
    const Matrix *A;
    int kind;
    bool anchor;
    int r0, r1;  // rows of subset t (all rows once plan_anchor has run)
    bool pair;   // the forward pass runs a pair of rows per wavefront
    FwdArgs fa;
    UpdateArgs u;
};
int plan_iteration(svr_recon *R, int t, IterPlan *p);
void end_iteration(svr_recon *R);

// Requests per batched launch (their arguments travel in the kernel
// arguments: about 100 B per forward item, 230 B per update item).
constexpr int BATCH_MAX = 8;

struct FwdItem {
    const int *row_ptr;
    const void *col;  // forward indices in tiled pixel order
    const void *val;
    FwdArgs a;
    int r0, r1;
    int pair;
    int blk0;  // first block of this item
};
struct FwdBatch {
    int n;
    int blocks;  // total blocks of the launch
    FwdItem it[BATCH_MAX];
};

struct UpdItem {
    const int *ptrT;
    const void *rowT;
    const void *valT;
    const float *sens_t;
    const double *sens;
    int N;
    int blk0;
    UpdateArgs u;
};
struct UpdBatch {
    int n;
    int blocks;
    UpdItem it[BATCH_MAX];
};

// SVREM anchors, batched the same way: plan_anchor turns an iteration plan at an anchor into the
// whole forward pass (p.fa, p.r0 = 0, p.r1 = M, p.pair; add_forward takes it) and the anchor's
// table and sums arguments; the table (one BP_G-lane group per (subset, pixel)) and the anchor
// sums + first update (a thread per pixel) then run as one launch each for several requests,
// through the device functions of the request's own anchor pass.
struct AncTabItem {
    const int *ptrT;
    const void *rowT;
    const void *valT;
    const int *row_start;
    int Ns, N;
    int blk0;
    SnapArgs a;
};
struct AncTabBatch {
    int n;
    int blocks;
    AncTabItem it[BATCH_MAX];
};
struct AncSumItem {
    const float *sens_t;
    const double *sens;
    int Ns, N;
    int blk0;
    SnapArgs a;
    UpdateArgs u;
};
struct AncSumBatch {
    int n;
    int blocks;
    AncSumItem it[BATCH_MAX];
};
int plan_anchor(svr_recon *R, IterPlan &p, SnapArgs *sa);
void add_anchor_table(AncTabBatch &b, const IterPlan &p, const SnapArgs &sa);
void add_anchor_sum(AncSumBatch &b, const IterPlan &p, const SnapArgs &sa);
int launch_anchor_table_batch(const Matrix &types, const AncTabBatch &b, hipStream_t s);
int launch_anchor_sum_batch(const AncSumBatch &b, hipStream_t s);

// Appends the plan's forward (update) work to the batch; the matrices of one
// batch share their weight and index types.
void add_forward(FwdBatch &b, const IterPlan &p);
void add_update(UpdBatch &b, const IterPlan &p);
// Launch the batch (types from `types`, a matrix of the batch); SVREM updates.
int launch_forward_batch(const Matrix &types, const FwdBatch &b, hipStream_t s);
int launch_update_batch(const Matrix &types, const UpdBatch &b, hipStream_t s);

// The objective in two halves, so that several recons' objectives share one wait:
// objective_enqueue enqueues the reductions on s and the copies of their results into *out
// (pinned host memory for an asynchronous copy); once s has completed, objective_result turns
// them into the objective, with the errors of svr_objective.
struct ObjectiveHost {
    double sums[2];  // log-likelihood, penalty sum
    int bad;         // entries outside the likelihood's domain
    int status;      // persistent-kernel abort flag
};
int objective_enqueue(svr_recon *R, hipStream_t s, ObjectiveHost *out);
int objective_result(svr_recon *R, const ObjectiveHost &o, hipStream_t s, double *phi);
// The current image of a single-slice recon (device, N floats).
const float *current_image(const svr_recon *R);

}  // namespace svr
