// Autotuner for the run lengths of the whole-matrix passes: pairs of rows of
// A per wavefront in the forward projection over every row (the anchor pass,
// the objective, svr_project over all subsets) and (subset, pixel) rows per
// lane group in the anchor table.  Each candidate is timed with HIP events on the
// matrix itself, on synthetic operands (image 1, data 1, background 0.1); the
// fastest is kept in the matrix.  The run length changes only which
// wavefront computes a row, never the row's arithmetic, so every result is
// bitwise the same under any tuning.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "trace.h"

namespace svr {
int forward_run_length(const Matrix &A, int rows);
int table_run_length(const Matrix &A);

namespace {

__global__ void k_fill(float *x, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = v;
}

int fill(float *x, int64_t n, float v, hipStream_t s) {
    k_fill<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, n, v);
    SVR_HIP(hipGetLastError());
    return SVR_OK;
}

// The per-subset passes of an epoch call, timed as an epoch runs them: the
// forward + ratio of subset t (one row per wavefront unless the subset is a
// pair pass) then its SVREM update, for t = 0 .. Ns-1, with HIP events around
// the whole sequence (median of 9 after one warm-up), for each pair of
// candidate batch widths.  Synthetic operands: image 1 (tiled and natural),
// data 1, background 0.1, statistics 0, table 1; the outputs go to scratch.
// A width never changes a result, only which loads are in flight together;
// the defaults (8, 5) are kept unless a pair is at least 2% faster, so that
// timing noise between near-equal widths does not move the choice.
int tune_subsets(Matrix &A, hipStream_t s, const FwdArgs &fa, float *f, float *table, float *fo, float *fto,
                 double *sd, hipEvent_t e0, hipEvent_t e1, int *best_fu, int *best_bu) {
    const int keep_fu = A.sub_fwd_u, keep_bu = A.sub_bp_u;
    bool single = false;  // any subset pass with one row per wavefront
    for (int t = 0; t < A.Ns; ++t) single = single || !forward_pairs_for(A.rows_of(t), A.pair_rows_eff());
    UpdateArgs u{};
    u.Ns = A.Ns;
    u.f = f;
    u.f_out = fo;
    u.ft_out = fto;
    u.tx = A.tx;
    u.alpha = 0.5;
    u.s_hat = sd;
    u.s_anc = sd + A.N;
    u.table = table;
    u.t2 = -1;
    u.pen = PenaltyArgs{SVR_PEN_QUADRATIC, 1.0, 1e-2, A.geom.nx, A.geom.ny};
    auto epoch_us = [&](float *out_us) -> int {
        std::vector<float> v;
        for (int r = 0; r < 10; ++r) {
            SVR_HIP(hipEventRecord(e0, s));
            for (int t = 0; t < A.Ns; ++t) {
                int q = launch_forward(A, A.row_start[t], A.row_start[t + 1], 1, fa, s);
                u.t = t;
                u.ratio = fa.out + A.row_start[t];
                if (!q) q = launch_update(A, UPD_SVREM, u, s);
                if (q) return q;
            }
            SVR_HIP(hipEventRecord(e1, s));
            SVR_HIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            SVR_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (r > 0) v.push_back(ms);
        }
        std::sort(v.begin(), v.end());
        *out_us = 1e3f * v[v.size() / 2];
        return SVR_OK;
    };
    static const int fwd_widths[] = {FWD_U, 4, 6}, bp_widths[] = {BP_U, 3, 4, 6, 8};
    float base = 0.0f, best = 0.0f;
    *best_fu = FWD_U;
    *best_bu = BP_U;
    int rc = SVR_OK;
    for (int fu : fwd_widths) {
        if (!single && fu != FWD_U) continue;
        for (int bu : bp_widths) {
            A.sub_fwd_u = fu;
            A.sub_bp_u = bu;
            float us = 0.0f;
            rc = epoch_us(&us);
            if (rc) break;
            if (fu == FWD_U && bu == BP_U) {
                base = best = us;
            } else if (us < best && us <= 0.98f * base) {
                best = us;
                *best_fu = fu;
                *best_bu = bu;
            }
        }
        if (rc) break;
    }
    A.sub_fwd_u = keep_fu;
    A.sub_bp_u = keep_bu;
    return rc;
}

int tune(Matrix &A, hipStream_t s, svr_tuning_t *out) {
    AllocStream as(s);
    float *f = nullptr, *g = nullptr, *w = nullptr, *ratio = nullptr, *table = nullptr, *fo = nullptr,
          *fto = nullptr;
    double *sd = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
    auto cleanup = [&]() {
        dfree(f); dfree(g); dfree(w); dfree(ratio); dfree(table); dfree(fo); dfree(fto); dfree(sd);
        for (hipEvent_t e : {e0, e1, e2, e3})
            if (e) (void)hipEventDestroy(e);
    };
    const int64_t NT = (int64_t)A.Ns * A.N;
    const int64_t NF = std::max<int64_t>(A.N, A.Nt);  // the forward reads the tiled order
    if (dalloc(&f, NF) != hipSuccess || dalloc(&g, A.M) != hipSuccess || dalloc(&w, A.M) != hipSuccess ||
        dalloc(&ratio, A.M) != hipSuccess || dalloc(&table, NT) != hipSuccess || dalloc(&fo, A.N) != hipSuccess ||
        dalloc(&fto, A.Nt) != hipSuccess || dalloc(&sd, 2 * (int64_t)A.N) != hipSuccess) {
        cleanup();
        set_error("tuning buffers: allocation failed");
        return SVR_ENOMEM;
    }
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess || hipEventCreate(&e2) != hipSuccess ||
        hipEventCreate(&e3) != hipSuccess) {
        cleanup();
        set_error("tuning: event creation failed");
        return SVR_EDEVICE;
    }
    int rc = fill(f, NF, 1.0f, s);
    if (!rc) rc = fill(table, NT, 1.0f, s);
    if (!rc && hipMemsetAsync(sd, 0, sizeof(double) * 2 * A.N, s) != hipSuccess) rc = SVR_EDEVICE;
    if (!rc) rc = fill(g, A.M, 1.0f, s);
    if (!rc) rc = fill(w, A.M, 0.1f, s);
    const int keep_f = A.run_fwd, keep_b = A.run_bp;
    FwdArgs fa{f, g, w, ratio, nullptr, nullptr};
    SnapArgs sa{};
    sa.ratio_all = ratio;
    sa.f = f;
    sa.table = table;
    // The two kernels are timed as the anchor pass runs them, alternately
    // (each streams its own layout of A, so each starts with the cache state
    // the other leaves behind): first the forward candidates with the table at
    // one row per group, then the table candidates after the chosen forward.
    auto pair_time = [&](double *us_fwd, double *us_tab) -> int {
        std::vector<float> tf, tt;
        for (int r = 0; r < 10; ++r) {
            SVR_HIP(hipEventRecord(e0, s));
            int q = launch_forward(A, 0, A.M, 1, fa, s);
            if (q) return q;
            SVR_HIP(hipEventRecord(e1, s));
            SVR_HIP(hipEventRecord(e2, s));
            q = launch_anchor_table(A, UPD_SVREM, sa, s);
            if (q) return q;
            SVR_HIP(hipEventRecord(e3, s));
            SVR_HIP(hipEventSynchronize(e3));
            float a = 0.0f, b = 0.0f;
            SVR_HIP(hipEventElapsedTime(&a, e0, e1));
            SVR_HIP(hipEventElapsedTime(&b, e2, e3));
            if (r > 0) {  // the first pair warms up
                tf.push_back(a);
                tt.push_back(b);
            }
        }
        std::sort(tf.begin(), tf.end());
        std::sort(tt.begin(), tt.end());
        *us_fwd = 1e3 * (double)tf[tf.size() / 2];
        *us_tab = 1e3 * (double)tt[tt.size() / 2];
        return SVR_OK;
    };
    int best_f = 1, best_b = 1;
    double us_f = 1e30, us_b = 1e30;
    A.run_bp = 1;
    for (int R : {1, 2, 3, 4, 6, 8, 12, 16}) {
        if (rc) break;
        if (R > 1 && ((int64_t)A.M + 1) / 2 < (int64_t)R * std::max(A.cus, 1) * 4) break;  // fewer waves than SIMDs
        A.run_fwd = R;
        double uf = 0.0, ut = 0.0;
        rc = pair_time(&uf, &ut);
        if (!rc && uf < us_f) { us_f = uf; best_f = R; }
    }
    A.run_fwd = best_f;
    for (int T : {1, 2, 3, 4, 6, 8, 12, 16}) {
        if (rc) break;
        if (T > 1 && NT < (int64_t)T * std::max(A.cus, 1) * 4 * (64 / BP_G)) break;
        A.run_bp = T;
        double uf = 0.0, ut = 0.0;
        rc = pair_time(&uf, &ut);
        if (!rc && ut < us_b) { us_b = ut; best_b = T; }
    }
    int best_fu = 0, best_bu = 0;
    if (!rc) {
        A.run_fwd = best_f;
        A.run_bp = best_b;
        rc = tune_subsets(A, s, fa, f, table, fo, fto, sd, e0, e1, &best_fu, &best_bu);
    }
    if (rc) {
        A.run_fwd = keep_f;
        A.run_bp = keep_b;
    } else {
        A.sub_fwd_u = best_fu;
        A.sub_bp_u = best_bu;
        if (out) {
            out->fwd_pairs_per_wave = best_f;
            out->bp_rows_per_group = best_b;
            out->fwd_pair_rows = A.pair_rows_eff();
            out->fwd_us = us_f;
            out->bp_us = us_b;
            out->fwd_natural_order = A.xcd_bands ? 0 : 1;
            out->subset_fwd_batch = best_fu;
            out->subset_bp_batch = best_bu;
        }
    }
    SVR_HIP(hipStreamSynchronize(s));
    cleanup();
    return rc;
}

// ---- tuning cache (environment SVR_TUNE_CACHE = a file path) --------------------
// One line per tuned matrix:
// "svr-tune 2 <key> fwd <R> bp <T> fu <U> bu <V> fwd_us <x> bp_us <y>",
// the key naming everything the timings depend on (geometry, subsets, weight
// and index types, device name and compute units).  A tune call whose key is
// in the file applies the stored choices without timing; otherwise it
// tunes and appends a line.  Lines that do not parse are ignored.
std::string cache_key(const Matrix &A) {
    hipDeviceProp_t prop{};
    std::string dev = "unknown";
    if (hipGetDeviceProperties(&prop, A.device) == hipSuccess) {
        dev = prop.gcnArchName;
        for (char &c : dev)
            if (c == ' ') c = '_';
    }
    const svr_geometry &g = A.geom;
    char buf[512];
    snprintf(buf, sizeof buf, "%dx%d/%.9g/%dx%d/%.9g/%.9g/ns%d/w%d/i%d/%s/cu%d", g.nx, g.ny, g.pixel_mm, g.n_views,
             g.n_bins, g.bin_mm, g.arc_rad, A.Ns, A.wtype, A.idx16 ? 16 : 32, dev.c_str(), A.cus);
    return buf;
}

bool valid_fwd_u(int U) { return U == 0 || U == 4 || U == 6 || U == 8; }
bool valid_bp_u(int U) { return U == 0 || U == 3 || U == 4 || U == 5 || U == 6 || U == 8; }

struct Cached {
    int fwd = 0, bp = 0, fu = 0, bu = 0;
    double fwd_us = 0.0, bp_us = 0.0;
};

bool cache_lookup(const char *path, const std::string &key, Cached *c) {
    FILE *fp = fopen(path, "r");
    if (!fp) return false;
    char line[1024], k[600];
    bool found = false;
    while (fgets(line, sizeof line, fp)) {
        int ver = 0;
        Cached e;
        if (sscanf(line, "svr-tune %d %599s fwd %d bp %d fu %d bu %d fwd_us %lf bp_us %lf", &ver, k, &e.fwd, &e.bp,
                   &e.fu, &e.bu, &e.fwd_us, &e.bp_us) == 8 &&
            ver == 2 && key == k && e.fwd >= 1 && e.fwd <= 31 && e.bp >= 1 && e.bp <= 1024 && valid_fwd_u(e.fu) &&
            valid_bp_u(e.bu)) {
            *c = e;  // the last matching line wins
            found = true;
        }
    }
    fclose(fp);
    return found;
}

void cache_store(const char *path, const std::string &key, const svr_tuning_t &t) {
    FILE *fp = fopen(path, "a");
    if (!fp) return;  // a cache that cannot be written only costs the next call its timing
    fprintf(fp, "svr-tune 2 %s fwd %d bp %d fu %d bu %d fwd_us %.3f bp_us %.3f\n", key.c_str(), t.fwd_pairs_per_wave,
            t.bp_rows_per_group, t.subset_fwd_batch, t.subset_bp_batch, t.fwd_us, t.bp_us);
    fclose(fp);
}

int tune_cached(Matrix &A, hipStream_t s, svr_tuning_t *out) {
    const char *path = getenv("SVR_TUNE_CACHE");
    if (!path || !*path) return tune(A, s, out);
    const std::string key = cache_key(A);
    Cached c;
    if (cache_lookup(path, key, &c)) {
        A.run_fwd = c.fwd;
        A.run_bp = c.bp;
        A.sub_fwd_u = c.fu;
        A.sub_bp_u = c.bu;
        if (out) {
            out->fwd_pairs_per_wave = c.fwd;
            out->bp_rows_per_group = c.bp;
            out->fwd_pair_rows = A.pair_rows_eff();
            out->fwd_us = c.fwd_us;
            out->bp_us = c.bp_us;
            out->fwd_natural_order = A.xcd_bands ? 0 : 1;
            out->subset_fwd_batch = c.fu;
            out->subset_bp_batch = c.bu;
        }
        return SVR_OK;
    }
    svr_tuning_t t{};
    const int rc = tune(A, s, &t);
    if (rc) return rc;
    cache_store(path, key, t);
    if (out) *out = t;
    return SVR_OK;
}

}  // namespace
}  // namespace svr

extern "C" {

int svr_matrix_get_tuning(const svr_matrix *A, svr_tuning_t *t) {
    svr::clear_error();
    SVR_REQUIRE(A && t, "NULL argument");
    t->fwd_pairs_per_wave = A->run_fwd > 0 ? A->run_fwd : svr::forward_run_length(*A, A->M);
    t->bp_rows_per_group = svr::table_run_length(*A);
    t->fwd_pair_rows = A->pair_rows_eff();
    t->fwd_us = 0.0;
    t->bp_us = 0.0;
    t->fwd_natural_order = A->xcd_bands ? 0 : 1;
    t->subset_fwd_batch = A->sub_fwd_u ? A->sub_fwd_u : svr::FWD_U;
    t->subset_bp_batch = A->sub_bp_u ? A->sub_bp_u : svr::BP_U;
    return SVR_OK;
}

int svr_matrix_set_tuning(svr_matrix *A, const svr_tuning_t *t) {
    svr::clear_error();
    SVR_REQUIRE(A && t, "NULL argument");
    SVR_REQUIRE(t->fwd_pairs_per_wave >= 0 && t->fwd_pairs_per_wave <= 31, "fwd_pairs_per_wave must be in [0, 31]");
    SVR_REQUIRE(t->bp_rows_per_group >= 0 && t->bp_rows_per_group <= 1024, "bp_rows_per_group must be in [0, 1024]");
    SVR_REQUIRE(t->fwd_pair_rows >= 0, "fwd_pair_rows must be >= 0");
    SVR_REQUIRE(t->fwd_natural_order == 0 || t->fwd_natural_order == 1, "fwd_natural_order must be 0 or 1");
    SVR_REQUIRE(svr::valid_fwd_u(t->subset_fwd_batch), "subset_fwd_batch must be 0, 4, 6 or 8");
    SVR_REQUIRE(svr::valid_bp_u(t->subset_bp_batch), "subset_bp_batch must be 0, 3, 4, 5, 6 or 8");
    A->sub_fwd_u = t->subset_fwd_batch;
    A->sub_bp_u = t->subset_bp_batch;
    A->xcd_bands = t->fwd_natural_order ? 0 : 1;
    A->run_fwd = t->fwd_pairs_per_wave;
    A->pair_rows = t->fwd_pair_rows;
    A->run_bp = t->bp_rows_per_group;
    return SVR_OK;
}

int svr_matrix_tune(svr_matrix *A, void *stream, svr_tuning_t *out) {
    svr::clear_error();
    svr::TraceRange tr("svr.tune");
    SVR_REQUIRE(A, "NULL argument");
    SVR_HIP(hipSetDevice(A->device));
    return svr::tune_cached(*A, (hipStream_t)stream, out);
}

}  // extern "C"
