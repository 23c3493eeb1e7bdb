// Continuous-batching server for independent SVREM reconstructions.
//
// Requests queue at submit; each scheduler tick enqueues one epoch of subset
// updates for every resident request (batched: one forward and one update
// launch per iteration for all requests of the same storage types; else each
// request on one of the server's streams), then admits queued requests (FIFO)
// while a slot is free and their device footprint fits the memory budget.
// The admissions of a tick run on a pool of host threads (up to 16), so their
// matrix builds (which wait on the host for their sizes) and initial epochs
// overlap each other and the enqueued epochs; requests of one geometry,
// subset count and weight type share one matrix, built once.  A request's
// kernels write only its own buffers and every reduction has a fixed order,
// so its result is the same whichever requests share the device (or its
// matrix) with it.  Finished requests hand their blocks to the server's block
// cache and their matrix, once unused, stays idle for later requests of its
// key; both give way when an admission needs the room in the budget.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <new>
#include <thread>
#include <tuple>
#include <utility>
#include <vector>

#include "batch.h"
#include "common.h"
#include "trace.h"
#include "util.h"

namespace {

using clk = std::chrono::steady_clock;

double ms_since(clk::time_point a, clk::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// SplitMix64 (Steele, Lea, Flood 2014): the request's subset sequence
struct SplitMix64 {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    int32_t below(int32_t n) { return (int32_t)(((next() >> 32) * (uint64_t)n) >> 32); }
};

enum State { QUEUED, RESIDENT, DONE };

// Requests with the same geometry, subset count and weight type share one matrix.
struct MatrixKey {
    int nx, ny, n_views, n_bins, n_subsets, wtype;
    double pixel_mm, bin_mm, arc_rad;
    bool operator<(const MatrixKey &o) const {
        return std::tie(nx, ny, n_views, n_bins, n_subsets, wtype, pixel_mm, bin_mm, arc_rad) <
               std::tie(o.nx, o.ny, o.n_views, o.n_bins, o.n_subsets, o.wtype, o.pixel_mm, o.bin_mm, o.arc_rad);
    }
};
MatrixKey key_of(const svr_serve_request &r) {
    const svr_geometry &g = r.geom;
    return MatrixKey{g.nx, g.ny, g.n_views, g.n_bins, r.n_subsets, r.wtype, g.pixel_mm, g.bin_mm, g.arc_rad};
}

// A matrix on the device and the resident requests that use it.  While refs > 0 its bytes are
// in used_bytes; at refs == 0 it stays on the device (idle, in idle_matrix_bytes) for later
// requests of its key until the budget needs the room.  Without sharing every request has an
// entry of its own, outside the index.
struct SharedMatrix {
    MatrixKey key{};
    bool indexed = false;     // in the server's index by key (sharing on)
    svr_matrix *A = nullptr;  // null until its build has succeeded
    int refs = 0;
    int64_t bytes = 0;        // the estimate until the build, then what the matrix holds
    int64_t built_bytes = 0;  // written by the build
    int build_rc = SVR_OK;
    int64_t last_tick = 0;
};

struct Request {
    uint64_t ticket = 0;
    svr_serve_request req{};
    std::vector<float> g, w;
    State state = QUEUED;
    int status = SVR_OK;
    int64_t est_bytes = 0, est_matrix = 0, held_bytes = 0;
    svr_matrix *A = nullptr;
    SharedMatrix *shared = nullptr;  // the server's entry for A (A is the entry's)
    bool builds = false;                    // this admission builds the entry's matrix
    svr_recon *R = nullptr;
    float *d_g = nullptr, *d_w = nullptr, *d_f0 = nullptr;
    int stream = 0;
    int epochs_done = 0;
    SplitMix64 rng{0};
    std::vector<float> f;
    double phi = 0.0;
    clk::time_point t_submit, t_admit, t_done;
};

// Device bytes a request will hold: the matrix (both layouts) and the recon.
// The matrix part is estimated from the geometry before the build: in parallel
// beam each view crosses about (1 + |cos| + |sin|) * pixel/bin pieces per
// pixel, 2.27 on average over angles; 2.6 leaves head room.
struct Footprint {
    int64_t matrix, rest;
};
Footprint footprint_estimate(const svr_serve_request &r) {
    const int64_t N = (int64_t)r.geom.nx * r.geom.ny;
    const int64_t M = (int64_t)r.geom.n_views * r.geom.n_bins;
    const int64_t Ns = r.n_subsets;
    const double ratio = std::max(1.0, r.geom.pixel_mm / r.geom.bin_mm);
    const int64_t nnz = (int64_t)(2.6 * ratio * (double)r.geom.n_views * (double)N);
    const int wb = r.wtype == SVR_W_F32 ? 4 : 2;
    Footprint fp;
    fp.matrix = 2 * nnz * (4 + wb) + 4 * (2 * M + Ns * N) + 4 * Ns * N + 8 * N;
    fp.rest = 4 * (3 * M + 2 * N) + 8 * (2 * N) + 4 * Ns * N + 8 * (M + N / 256 + 8) + 4 * (2 * M + N);
    return fp;
}

}  // namespace

struct svr_server {
    svr_serve_config cfg{};
    std::vector<hipStream_t> streams;
    std::map<uint64_t, std::unique_ptr<Request>> reqs;
    std::deque<uint64_t> queue;
    std::vector<uint64_t> resident;
    uint64_t next_ticket = 1;
    int64_t used_bytes = 0;
    int device = 0;
    int64_t ticks = 0, admitted = 0, completed = 0, epochs = 0;  // running totals (svr_serve_stats)
    // the device blocks of finished requests, kept for the requests admitted later (within the
    // memory budget together with used_bytes)
    svr::BlockCache cache;
    std::list<SharedMatrix> mats;                   // every matrix entry (stable addresses)
    std::map<MatrixKey, SharedMatrix *> mat_index;  // the shared ones, by key
    int64_t idle_matrix_bytes = 0;
    int64_t matrix_reuses = 0;
    char *pin = nullptr;  // pinned staging for the results of the requests finishing in a tick
    size_t pin_bytes = 0;
};

using namespace svr;

namespace {

// Destroys the entry's matrix (blocks kept in the server's cache when keep) and drops the entry.
void destroy_matrix_entry(svr_server *S, SharedMatrix *m, bool keep) {
    BlockCacheScope sc(&S->cache, keep);
    if (m->A) svr_matrix_destroy(m->A);
    if (m->indexed) S->mat_index.erase(m->key);
    for (auto it = S->mats.begin(); it != S->mats.end(); ++it)
        if (&*it == m) {
            S->mats.erase(it);
            break;
        }
}

// Drops q's use of its matrix; the last user's drop leaves the matrix idle (kept for later
// requests of its key) or, without sharing, destroys it.
void unref_matrix(svr_server *S, Request *q, bool keep) {
    SharedMatrix *m = q->shared;
    q->shared = nullptr;
    q->A = nullptr;
    if (!m || --m->refs > 0) return;
    S->used_bytes -= m->bytes;
    if (keep && m->indexed && m->A) {
        m->last_tick = S->ticks;
        S->idle_matrix_bytes += m->bytes;
    } else {
        destroy_matrix_entry(S, m, keep);
    }
}

// Destroys the least recently used idle matrix other than `except` (its blocks go to the block
// cache); false if there is none.
bool evict_idle_matrix(svr_server *S, const SharedMatrix *except) {
    SharedMatrix *lru = nullptr;
    for (SharedMatrix &m : S->mats)
        if (m.refs == 0 && m.A && &m != except && (!lru || m.last_tick < lru->last_tick)) lru = &m;
    if (!lru) return false;
    S->idle_matrix_bytes -= lru->bytes;
    destroy_matrix_entry(S, lru, true);
    return true;
}

// Frees q's device objects.  keep: every stream has finished with them, and their blocks stay
// in the server's cache; else they are freed, stream-ordered on q's stream.
void release(svr_server *S, Request *q, bool keep) {
    TraceRange tr("svr.serve.release");
    BlockCacheScope sc(&S->cache, keep);
    if (q->R) svr_recon_destroy(q->R);
    unref_matrix(S, q, keep);
    AllocStream as(S->streams[q->stream]);
    dfree(q->d_g);
    dfree(q->d_w);
    dfree(q->d_f0);
    q->R = nullptr;
    q->A = nullptr;
    q->d_g = q->d_w = q->d_f0 = nullptr;
    S->used_bytes -= q->held_bytes;
    q->held_bytes = 0;
}

__global__ void k_fill(float *x, int64_t n, float v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

// Builds the matrix of the entry q->shared on q's stream and waits for it (requests on other
// streams use it next).  Touches the server only through its block cache (locked) and the
// entry, so several builds may run at once.
int build_shared(svr_server *S, Request *q, hipStream_t s) {
    TraceRange tr("svr.serve.build");
    AllocStream as(s);
    BlockCacheScope sc(&S->cache, false);
    const svr_serve_request &r = q->req;
    svr_matrix *A = nullptr;
    int rc = svr_build_system_matrix(&r.geom, r.n_subsets, r.wtype, nullptr, s, &A);
    if (rc) return rc;
    if (hipStreamSynchronize(s) != hipSuccess) {
        svr_matrix_destroy(A);
        set_error("matrix build failed on the device");
        return SVR_EDEVICE;
    }
    svr_matrix_info_t inf;
    svr_matrix_info(A, &inf, nullptr);
    q->shared->A = A;
    q->shared->built_bytes = inf.bytes;
    return SVR_OK;
}

// The request's recon on its (built) matrix and the OSEM initialisation epoch; touches the
// server only through its block cache (locked), so several admissions may run at once.
int admit(svr_server *S, Request *q, hipStream_t s) {
    TraceRange tr("svr.serve.admit");
    AllocStream as(s);
    BlockCacheScope sc(&S->cache, false);
    const svr_serve_request &r = q->req;
    const int64_t M = (int64_t)r.geom.n_views * r.geom.n_bins;
    const int64_t N = (int64_t)r.geom.nx * r.geom.ny;
    int rc = SVR_OK;
    SVR_HIP(dalloc(&q->d_g, M));
    SVR_HIP(dalloc(&q->d_w, M));
    SVR_HIP(dalloc(&q->d_f0, N));
    SVR_HIP(hipMemcpyAsync(q->d_g, q->g.data(), sizeof(float) * M, hipMemcpyHostToDevice, s));
    SVR_HIP(hipMemcpyAsync(q->d_w, q->w.data(), sizeof(float) * M, hipMemcpyHostToDevice, s));
    k_fill<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(q->d_f0, N, r.f0_value);
    SVR_HIP(hipGetLastError());
    rc = svr_recon_create(q->A, q->d_g, q->d_w, q->d_f0, 1, &r.params, s, &q->R);
    if (rc) return rc;
    std::vector<int32_t> cyc(r.n_subsets);
    for (int t = 0; t < r.n_subsets; ++t) cyc[t] = t;
    rc = svr_osem_epoch(q->R, cyc.data(), r.n_subsets, s);
    if (rc) return rc;
    q->rng.s = r.order_seed;
    q->t_admit = clk::now();
    q->state = RESIDENT;
    return SVR_OK;
}

// Runs fn(S, q, q's stream) for every request, on up to ADMIT_THREADS host threads that take
// the requests in turn: a matrix build waits on the host for its sizes, and several builds'
// waits (and their kernels, on different streams) then overlap.
constexpr size_t ADMIT_THREADS = 16;
void run_each(svr_server *S, const std::vector<Request *> &adm, std::vector<int> &rcs,
              int (*fn)(svr_server *, Request *, hipStream_t)) {
    rcs.assign(adm.size(), SVR_OK);
    if (adm.empty()) return;
    if (adm.size() == 1) {
        rcs[0] = fn(S, adm[0], S->streams[adm[0]->stream]);
        return;
    }
    std::atomic<size_t> next{0};
    auto work = [S, &adm, &rcs, &next, fn] {
        const bool on_device = hipSetDevice(S->device) == hipSuccess;
        for (size_t k; (k = next.fetch_add(1)) < adm.size();)
            rcs[k] = on_device ? fn(S, adm[k], S->streams[adm[k]->stream]) : SVR_EDEVICE;
    };
    std::vector<std::thread> th;
    const size_t n_threads = std::min(adm.size(), ADMIT_THREADS) - 1;  // and this one
    for (size_t k = 0; k < n_threads; ++k) {
        try {
            th.emplace_back(work);
        } catch (const std::exception &) {
            break;  // no more threads to be had: the ones running (and this one) take the rest
        }
    }
    work();
    for (std::thread &t : th) t.join();
}

// One epoch of every resident request with the subset iterations batched:
// for each iteration index, the requests at an anchor run as one whole-matrix
// forward, one table and one anchor-sums + update launch per group of requests
// with the same weight and index types, the others as one forward and one
// update launch per batch (the requests of one storage type, up to BATCH_MAX a
// batch); each batch's launches go to one stream, different batches' to
// different ones.
void batched_epoch(svr_server *S) {
    TraceRange tr("svr.serve.batched_epoch");
    // The requests of one storage type (weight type, index width) split into batches of up to
    // BATCH_MAX, fixed for the tick; each batch takes a stream of its own for the whole tick, so
    // a request's iterations stay in order while different batches' launches overlap.
    using BatchKey = std::pair<int, int>;  // storage type, the batch's index within its type
    struct Res {
        Request *q;
        std::vector<int32_t> order;
        BatchKey batch;
    };
    std::vector<Res> rs;
    std::map<int, int> per_type;
    std::map<BatchKey, int> stream_of_batch;
    int max_ns = 0;
    for (uint64_t tk : S->resident) {
        Request *q = S->reqs[tk].get();
        const int Ns = q->req.n_subsets;
        const Matrix &A = *q->A;
        const int type = A.wtype * 2 + A.idx16;
        Res r{q, std::vector<int32_t>(Ns), BatchKey(type, per_type[type]++ / BATCH_MAX)};
        for (int i = 0; i < Ns; ++i) r.order[i] = q->rng.below(Ns);
        if (!stream_of_batch.count(r.batch)) stream_of_batch[r.batch] = (int)stream_of_batch.size();
        max_ns = std::max(max_ns, Ns);
        rs.push_back(std::move(r));
    }
    auto stream_of = [&](const BatchKey &batch) { return S->streams[stream_of_batch[batch] % (int)S->streams.size()]; };
    for (int j = 0; j < max_ns; ++j) {
        std::map<BatchKey, std::vector<std::pair<Request *, IterPlan>>> groups, anchors;
        for (Res &r : rs) {
            Request *q = r.q;
            if (j >= (int)r.order.size() || q->status != SVR_OK) continue;
            IterPlan pl;
            int rc = plan_iteration(q->R, r.order[j], &pl);
            if (rc) {
                q->status = rc;
                continue;
            }
            (pl.anchor ? anchors : groups)[r.batch].push_back({q, pl});
        }
        // the requests at an anchor: the whole forward pass, the table and the anchor sums with
        // the first update, each one launch per group (up to BATCH_MAX requests)
        for (auto &kv : anchors) {
            auto &v = kv.second;
            for (size_t c = 0; c < v.size(); c += BATCH_MAX) {
                const size_t e = std::min(v.size(), c + BATCH_MAX);
                FwdBatch fb{};
                AncTabBatch tb{};
                AncSumBatch sb{};
                std::vector<Request *> in;
                for (size_t i = c; i < e; ++i) {
                    SnapArgs sa;
                    const int rc = plan_anchor(v[i].first->R, v[i].second, &sa);
                    if (rc) {
                        v[i].first->status = rc;
                        continue;
                    }
                    add_forward(fb, v[i].second);
                    add_anchor_table(tb, v[i].second, sa);
                    add_anchor_sum(sb, v[i].second, sa);
                    in.push_back(v[i].first);
                }
                const Matrix &types = *v[c].second.A;
                hipStream_t sg = stream_of(kv.first);
                int rc = launch_forward_batch(types, fb, sg);
                if (!rc) rc = launch_anchor_table_batch(types, tb, sg);
                if (!rc) rc = launch_anchor_sum_batch(sb, sg);
                if (rc)
                    for (Request *q : in) q->status = rc;
            }
            for (auto &qp : v) end_iteration(qp.first->R);
        }
        for (auto &kv : groups) {
            auto &v = kv.second;
            for (size_t c = 0; c < v.size(); c += BATCH_MAX) {
                const size_t e = std::min(v.size(), c + BATCH_MAX);
                FwdBatch fb{};
                for (size_t i = c; i < e; ++i) add_forward(fb, v[i].second);
                const int rc = launch_forward_batch(*v[c].second.A, fb, stream_of(kv.first));
                if (rc)
                    for (size_t i = c; i < e; ++i) v[i].first->status = rc;
            }
            for (size_t c = 0; c < v.size(); c += BATCH_MAX) {
                const size_t e = std::min(v.size(), c + BATCH_MAX);
                UpdBatch ub{};
                for (size_t i = c; i < e; ++i) add_update(ub, v[i].second);
                const int rc = launch_update_batch(*v[c].second.A, ub, stream_of(kv.first));
                if (rc)
                    for (size_t i = c; i < e; ++i) v[i].first->status = rc;
            }
            for (auto &qp : v) end_iteration(qp.first->R);
        }
    }
    for (Res &r : rs) r.q->epochs_done++;
    S->epochs += (int64_t)rs.size();
}

// One request's objective and image with waits of its own (when no pinned staging is to be had).
void finish_one(svr_server *S, Request *q, hipStream_t s) {
    const int64_t N = (int64_t)q->req.geom.nx * q->req.geom.ny;
    double phi = 0.0;
    int rc = svr_objective(q->R, &phi, s);
    q->phi = phi;
    q->status = rc;
    q->f.resize(N);
    float *tmp = nullptr;
    AllocStream as(s);
    if (dalloc(&tmp, N) == hipSuccess) {
        svr_get_image(q->R, tmp, s);
        (void)hipMemcpyAsync(q->f.data(), tmp, sizeof(float) * N, hipMemcpyDeviceToHost, s);
        (void)hipStreamSynchronize(s);
        dfree(tmp);
    } else {
        q->status = SVR_ENOMEM;
    }
    q->state = DONE;
    q->t_done = clk::now();
    release(S, q, true);  // every stream was synchronised before the request finished
}

// The requests finishing this tick: their objectives and image copies (into pinned staging)
// are enqueued on their streams, the streams waited for once, then the results read.
void finish_all(svr_server *S, const std::vector<Request *> &done) {
    if (done.empty()) return;
    TraceRange tr("svr.serve.finish");
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    auto n_of = [](const Request *q) { return (size_t)q->req.geom.nx * q->req.geom.ny; };
    size_t need = 0;
    for (const Request *q : done) need += al(sizeof(ObjectiveHost)) + al(sizeof(float) * n_of(q));
    if (need > S->pin_bytes) {
        if (S->pin) (void)hipHostFree(S->pin);
        S->pin = nullptr;
        const size_t cap = std::max(need, 2 * S->pin_bytes);
        S->pin_bytes = 0;
        if (hipHostMalloc((void **)&S->pin, cap) == hipSuccess) {
            S->pin_bytes = cap;
        } else {
            S->pin = nullptr;
            (void)hipGetLastError();
        }
    }
    if (!S->pin) {
        for (Request *q : done) finish_one(S, q, S->streams[q->stream]);
        return;
    }
    std::vector<ObjectiveHost *> oh(done.size());
    std::vector<float *> img(done.size());
    std::vector<int> rcs(done.size());
    char *p = S->pin;
    for (size_t k = 0; k < done.size(); ++k) {
        Request *q = done[k];
        hipStream_t s = S->streams[q->stream];
        oh[k] = reinterpret_cast<ObjectiveHost *>(p);
        p += al(sizeof(ObjectiveHost));
        img[k] = reinterpret_cast<float *>(p);
        p += al(sizeof(float) * n_of(q));
        *oh[k] = ObjectiveHost{};
        rcs[k] = objective_enqueue(q->R, s, oh[k]);
        const hipError_t e =
            hipMemcpyAsync(img[k], current_image(q->R), sizeof(float) * n_of(q), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess && !rcs[k]) {
            set_error("image copy failed: %s", hipGetErrorString(e));
            rcs[k] = SVR_EDEVICE;
        }
    }
    for (hipStream_t st : S->streams) (void)hipStreamSynchronize(st);
    for (size_t k = 0; k < done.size(); ++k) {
        Request *q = done[k];
        hipStream_t s = S->streams[q->stream];
        double phi = 0.0;
        int rc = rcs[k];
        if (!rc) {
            rc = objective_result(q->R, *oh[k], s, &phi);
            if (rc == SVR_EDEVICE) (void)hipStreamSynchronize(s);  // its flag reset is in flight
        }
        q->phi = phi;
        q->status = rc;
        q->f.assign(img[k], img[k] + n_of(q));
        q->state = DONE;
        q->t_done = clk::now();
        release(S, q, true);  // every stream has finished with it
    }
}

// Keeps the cache within what the budget leaves beside the resident requests.
void trim_cache(svr_server *S, int64_t room) {
    if (S->cache.idle_bytes <= room) return;
    AllocStream as(S->streams[0]);
    block_cache_trim(S->cache, std::max<int64_t>(room, 0));
}

// Idle matrices, then kept blocks, give way until what the server holds fits the budget.
void fit_budget(svr_server *S) {
    while (S->used_bytes + S->idle_matrix_bytes > S->cfg.mem_budget_bytes && evict_idle_matrix(S, nullptr)) {
    }
    trim_cache(S, S->cfg.mem_budget_bytes - S->used_bytes - S->idle_matrix_bytes);
}

}  // namespace

extern "C" {

int svr_serve_create(const svr_serve_config *cfg, svr_server **out) {
    clear_error();
    SVR_REQUIRE(cfg && out, "NULL argument");
    SVR_REQUIRE(cfg->mem_budget_bytes > 0 && cfg->max_slots >= 1 && cfg->n_streams >= 1,
                "mem_budget_bytes > 0, max_slots >= 1 and n_streams >= 1 are required");
    SVR_REQUIRE(cfg->batch == 0 || cfg->batch == 1, "batch must be 0 or 1");
    SVR_REQUIRE(cfg->share_matrices == 0 || cfg->share_matrices == 1, "share_matrices must be 0 or 1");
    *out = nullptr;
    svr_server *S = new (std::nothrow) svr_server();
    SVR_REQUIRE(S, "host allocation failed");
    S->cfg = *cfg;
    (void)hipGetDevice(&S->device);
    for (int i = 0; i < cfg->n_streams; ++i) {
        hipStream_t st;
        hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) {
            svr_serve_destroy(S);
            set_error("stream creation failed: %s", hipGetErrorString(e));
            return SVR_EDEVICE;
        }
        S->streams.push_back(st);
    }
    *out = S;
    return SVR_OK;
}

int svr_serve_submit(svr_server *S, const svr_serve_request *r, uint64_t *ticket) {
    clear_error();
    SVR_REQUIRE(S && r && ticket, "NULL argument");
    const svr_geometry &g = r->geom;
    SVR_REQUIRE(g.nx >= 1 && g.ny >= 1 && g.n_views >= 1 && g.n_bins >= 1 && g.pixel_mm > 0 && g.bin_mm > 0 &&
                    g.arc_rad > 0,
                "invalid geometry");
    SVR_REQUIRE(r->n_subsets >= 1 && r->n_subsets <= g.n_views, "n_subsets must be in [1, n_views]");
    SVR_REQUIRE(r->params.algo == SVR_ALGO_SVREM, "the server runs SVREM requests");
    SVR_REQUIRE(!(S->cfg.batch && (r->params.flags & SVR_FLAG_PERSISTENT_EPOCH)),
                "a batching server runs the per-phase kernels: SVR_FLAG_PERSISTENT_EPOCH is not available");
    SVR_REQUIRE(r->epochs >= 1, "epochs must be >= 1");
    SVR_REQUIRE(r->g_host && r->w_host, "g_host and w_host are required");
    SVR_REQUIRE(r->f0_value > 0 && std::isfinite(r->f0_value), "f0_value must be finite and > 0");
    auto q = std::make_unique<Request>();
    q->req = *r;
    const int64_t M = (int64_t)g.n_views * g.n_bins;
    q->g.assign(r->g_host, r->g_host + M);
    q->w.assign(r->w_host, r->w_host + M);
    q->req.g_host = nullptr;
    q->req.w_host = nullptr;
    const Footprint fp = footprint_estimate(*r);
    q->est_bytes = fp.matrix + fp.rest;
    q->est_matrix = fp.matrix;
    if (q->est_bytes > S->cfg.mem_budget_bytes) {
        set_error("request needs about %lld bytes, more than the server budget %lld", (long long)q->est_bytes,
                  (long long)S->cfg.mem_budget_bytes);
        return SVR_EINVAL;
    }
    q->ticket = S->next_ticket++;
    q->t_submit = clk::now();
    *ticket = q->ticket;
    S->queue.push_back(q->ticket);
    S->reqs[q->ticket] = std::move(q);
    return SVR_OK;
}

int svr_serve_step(svr_server *S, int32_t max_ticks) {
    clear_error();
    TraceRange tr("svr.serve_step");
    SVR_REQUIRE(S, "NULL server");
    SVR_HIP(hipSetDevice(S->device));
    for (int tick = 0; max_ticks <= 0 || tick < max_ticks; ++tick) {
        // one epoch of SVREM for every resident request: batched, or each
        // request's epoch on its own stream, overlapped over streams
        const size_t running = S->resident.size();
        if (S->cfg.batch) {
            batched_epoch(S);
        } else {
            for (uint64_t tk : S->resident) {
                Request *q = S->reqs[tk].get();
                const int Ns = q->req.n_subsets;
                std::vector<int32_t> order(Ns);
                for (int i = 0; i < Ns; ++i) order[i] = q->rng.below(Ns);
                int rc = svr_svrem_epoch(q->R, order.data(), Ns, S->streams[q->stream]);
                if (rc) q->status = rc;
                q->epochs_done++;
            }
            S->epochs += (int64_t)running;
        }
        ++S->ticks;
        // admission, FIFO while a slot is free and the estimate fits the budget, after the epochs
        // are enqueued: a new request's matrix build (which waits on the host for its sizes) and
        // OSEM epoch then overlap the resident requests' epochs on the other streams
        std::vector<Request *> adm, builders;
        while (!S->queue.empty() && (int)(S->resident.size() + adm.size()) < S->cfg.max_slots) {
            Request *q = S->reqs[S->queue.front()].get();
            const MatrixKey key = key_of(q->req);
            SharedMatrix *m = nullptr;
            if (S->cfg.share_matrices) {
                auto it = S->mat_index.find(key);
                if (it != S->mat_index.end()) m = it->second;
            }
            // a matrix in use or idle costs nothing more; a new one its estimate
            const int64_t rest = q->est_bytes - q->est_matrix, need = rest + (m ? 0 : q->est_matrix);
            auto room = [&] { return S->cfg.mem_budget_bytes - S->used_bytes - S->idle_matrix_bytes - need; };
            while (room() < 0 && evict_idle_matrix(S, m)) {
            }
            if (room() < 0) break;
            trim_cache(S, room());
            S->queue.pop_front();
            q->stream = (int)(q->ticket % S->streams.size());
            q->held_bytes = rest;
            S->used_bytes += rest;
            if (m) {
                if (m->refs == 0 && m->A) {  // idle until now
                    S->idle_matrix_bytes -= m->bytes;
                    S->used_bytes += m->bytes;
                }
                ++S->matrix_reuses;
            } else {
                S->mats.emplace_back();
                m = &S->mats.back();
                m->key = key;
                m->bytes = q->est_matrix;  // reserved until the build tells the matrix's size
                S->used_bytes += m->bytes;
                if (S->cfg.share_matrices) {
                    S->mat_index[key] = m;
                    m->indexed = true;
                }
                q->builds = true;
                builders.push_back(q);
            }
            ++m->refs;
            q->shared = m;
            adm.push_back(q);
        }
        // the new matrices first (each on its builder's stream, waited for), then every admitted
        // request's recon and OSEM epoch on its own stream
        std::vector<int> brc, rcs(adm.size(), SVR_OK);
        run_each(S, builders, brc, build_shared);
        for (size_t k = 0; k < builders.size(); ++k) {
            SharedMatrix *m = builders[k]->shared;
            if (brc[k]) {
                m->build_rc = brc[k];
            } else {
                S->used_bytes += m->built_bytes - m->bytes;
                m->bytes = m->built_bytes;
            }
        }
        std::vector<Request *> ready;
        std::vector<size_t> ready_at;
        for (size_t k = 0; k < adm.size(); ++k) {
            Request *q = adm[k];
            if (!q->shared->A) {
                rcs[k] = q->shared->build_rc ? q->shared->build_rc : SVR_EDEVICE;
                continue;
            }
            q->A = q->shared->A;
            ready.push_back(q);
            ready_at.push_back(k);
        }
        std::vector<int> arc;
        run_each(S, ready, arc, admit);
        for (size_t k = 0; k < ready.size(); ++k) rcs[ready_at[k]] = arc[k];
        for (size_t k = 0; k < adm.size(); ++k) {
            Request *q = adm[k];
            ++S->admitted;
            if (rcs[k]) {
                q->status = rcs[k];
                q->state = DONE;
                q->t_admit = q->t_done = clk::now();
                // its stream may still run the failed admission's work, which reads the matrix
                (void)hipStreamSynchronize(S->streams[q->stream]);
                release(S, q, true);
                ++S->completed;
                continue;
            }
            S->resident.push_back(q->ticket);
        }
        fit_budget(S);  // matrices larger than estimated
        if (S->resident.empty()) return SVR_OK;
        {
            TraceRange ts("svr.serve.sync");
            for (hipStream_t st : S->streams) SVR_HIP(hipStreamSynchronize(st));
        }
        std::vector<uint64_t> still;
        std::vector<Request *> done;
        std::vector<int> prior;  // an error from the epochs outranks the objective's status
        for (size_t i = 0; i < S->resident.size(); ++i) {
            const uint64_t tk = S->resident[i];
            Request *q = S->reqs[tk].get();
            if (i < running && (q->status != SVR_OK || q->epochs_done >= q->req.epochs)) {
                done.push_back(q);
                prior.push_back(q->status);
            } else {
                still.push_back(tk);
            }
        }
        finish_all(S, done);
        for (size_t k = 0; k < done.size(); ++k) {
            if (prior[k] != SVR_OK) done[k]->status = prior[k];
            ++S->completed;
        }
        S->resident.swap(still);
        fit_budget(S);
        if (max_ticks <= 0 && S->resident.empty() && S->queue.empty()) return SVR_OK;
    }
    return SVR_OK;
}

int svr_serve_poll(svr_server *S, uint64_t ticket, svr_serve_result *res) {
    clear_error();
    SVR_REQUIRE(S && res, "NULL argument");
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
        set_error("unknown ticket %llu", (unsigned long long)ticket);
        return SVR_ENOTFOUND;
    }
    Request *q = it->second.get();
    if (q->state != DONE) return SVR_PENDING;
    if (res->f_host) {
        const size_t n = (size_t)q->req.geom.nx * q->req.geom.ny;
        if (q->f.size() == n)
            memcpy(res->f_host, q->f.data(), sizeof(float) * n);
        else
            memset(res->f_host, 0, sizeof(float) * n);  // cancelled, or failed before an image existed
    }
    res->phi = q->phi;
    res->queue_ms = ms_since(q->t_submit, q->t_admit);
    res->run_ms = ms_since(q->t_admit, q->t_done);
    res->status = q->status;
    S->reqs.erase(it);
    return SVR_OK;
}

int svr_serve_done(const svr_server *S, uint64_t *tickets, int32_t cap, int32_t *n) {
    clear_error();
    SVR_REQUIRE(S && n, "NULL argument");
    SVR_REQUIRE(cap >= 0 && (tickets || cap == 0), "cap must be >= 0, with a tickets array when > 0");
    int32_t k = 0;
    for (const auto &kv : S->reqs) {
        if (k >= cap) break;
        if (kv.second->state == DONE) tickets[k++] = kv.first;
    }
    *n = k;
    return SVR_OK;
}

int svr_serve_cancel(svr_server *S, uint64_t ticket) {
    clear_error();
    SVR_REQUIRE(S, "NULL server");
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
        set_error("unknown ticket %llu", (unsigned long long)ticket);
        return SVR_ENOTFOUND;
    }
    Request *q = it->second.get();
    if (q->state == DONE) return SVR_OK;
    if (q->state == QUEUED) {
        for (auto i = S->queue.begin(); i != S->queue.end(); ++i)
            if (*i == ticket) { S->queue.erase(i); break; }
        q->t_admit = clk::now();
    } else {
        for (hipStream_t st : S->streams) (void)hipStreamSynchronize(st);
        release(S, q, true);
        for (auto i = S->resident.begin(); i != S->resident.end(); ++i)
            if (*i == ticket) { S->resident.erase(i); break; }
    }
    q->state = DONE;
    q->status = SVR_ECANCELLED;
    q->t_done = clk::now();
    ++S->completed;
    return SVR_OK;
}

int svr_serve_trim(svr_server *S, int32_t drop_matrices, int64_t keep_bytes) {
    clear_error();
    TraceRange tr("svr.serve.trim");
    SVR_REQUIRE(S, "NULL server");
    SVR_REQUIRE(drop_matrices == 0 || drop_matrices == 1, "drop_matrices must be 0 or 1");
    SVR_REQUIRE(keep_bytes >= 0, "keep_bytes must be >= 0");
    SVR_HIP(hipSetDevice(S->device));
    if (drop_matrices)
        while (evict_idle_matrix(S, nullptr)) {
        }
    trim_cache(S, keep_bytes);
    return SVR_OK;
}

int svr_serve_stats(const svr_server *S, svr_serve_stats_t *out) {
    clear_error();
    SVR_REQUIRE(S && out, "NULL argument");
    int32_t done = 0;
    for (const auto &kv : S->reqs) done += kv.second->state == DONE ? 1 : 0;
    out->queued = (int32_t)S->queue.size();
    out->resident = (int32_t)S->resident.size();
    out->max_slots = S->cfg.max_slots;
    out->done_unpolled = done;
    out->used_bytes = S->used_bytes;
    out->cached_bytes = S->cache.idle_bytes + S->idle_matrix_bytes;
    out->block_reuses = S->cache.reuses;
    out->matrix_reuses = S->matrix_reuses;
    out->mem_budget_bytes = S->cfg.mem_budget_bytes;
    out->ticks = S->ticks;
    out->admitted = S->admitted;
    out->completed = S->completed;
    out->epochs = S->epochs;
    return SVR_OK;
}

void svr_serve_destroy(svr_server *S) {
    if (!S) return;
    (void)hipSetDevice(S->device);
    for (hipStream_t st : S->streams) (void)hipStreamSynchronize(st);
    for (auto &kv : S->reqs) release(S, kv.second.get(), true);
    while (!S->mats.empty()) {  // the idle matrices
        S->idle_matrix_bytes -= S->mats.front().bytes;
        destroy_matrix_entry(S, &S->mats.front(), true);
    }
    if (!S->streams.empty()) {
        trim_cache(S, 0);
        (void)hipStreamSynchronize(S->streams[0]);
    }
    for (hipStream_t st : S->streams) (void)hipStreamDestroy(st);
    if (S->pin) (void)hipHostFree(S->pin);
    delete S;
}

}  // extern "C"
