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

int tune(Matrix &A, hipStream_t s, svr_tuning_t *out) {
    AllocStream as(s);
    float *f = nullptr, *g = nullptr, *w = nullptr, *ratio = nullptr, *table = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
    auto cleanup = [&]() {
        dfree(f); dfree(g); dfree(w); dfree(ratio); dfree(table);
        for (hipEvent_t e : {e0, e1, e2, e3})
            if (e) (void)hipEventDestroy(e);
    };
    const int64_t NT = (int64_t)A.Ns * A.N;
    const int64_t NF = std::max<int64_t>(A.N, A.Nt);  // the forward reads the tiled order
    if (dalloc(&f, NF) != hipSuccess || dalloc(&g, A.M) != hipSuccess || dalloc(&w, A.M) != hipSuccess ||
        dalloc(&ratio, A.M) != hipSuccess || dalloc(&table, NT) != hipSuccess) {
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
    if (rc) {
        A.run_fwd = keep_f;
        A.run_bp = keep_b;
    } else {
        A.run_fwd = best_f;
        A.run_bp = best_b;
        if (out) {
            out->fwd_pairs_per_wave = best_f;
            out->bp_rows_per_group = best_b;
            out->fwd_pair_rows = A.pair_rows_eff();
            out->fwd_us = us_f;
            out->bp_us = us_b;
            out->fwd_natural_order = A.xcd_bands ? 0 : 1;
        }
    }
    SVR_HIP(hipStreamSynchronize(s));
    cleanup();
    return rc;
}

// ---- tuning cache (environment SVR_TUNE_CACHE = a file path) --------------------
// One line per tuned matrix: "svr-tune 1 <key> fwd <R> bp <T> fwd_us <x> bp_us <y>",
// the key naming everything the timings depend on (geometry, subsets, weight
// and index types, device name and compute units).  A tune call whose key is
// in the file applies the stored run lengths without timing; otherwise it
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

bool cache_lookup(const char *path, const std::string &key, int *fwd, int *bp, double *fwd_us, double *bp_us) {
    FILE *fp = fopen(path, "r");
    if (!fp) return false;
    char line[1024], k[600];
    bool found = false;
    while (fgets(line, sizeof line, fp)) {
        int ver = 0, R = 0, T = 0;
        double uf = 0.0, ub = 0.0;
        if (sscanf(line, "svr-tune %d %599s fwd %d bp %d fwd_us %lf bp_us %lf", &ver, k, &R, &T, &uf, &ub) == 6 &&
            ver == 1 && key == k && R >= 1 && R <= 31 && T >= 1 && T <= 1024) {
            *fwd = R;  // the last matching line wins
            *bp = T;
            *fwd_us = uf;
            *bp_us = ub;
            found = true;
        }
    }
    fclose(fp);
    return found;
}

void cache_store(const char *path, const std::string &key, int fwd, int bp, double fwd_us, double bp_us) {
    FILE *fp = fopen(path, "a");
    if (!fp) return;  // a cache that cannot be written only costs the next call its timing
    fprintf(fp, "svr-tune 1 %s fwd %d bp %d fwd_us %.3f bp_us %.3f\n", key.c_str(), fwd, bp, fwd_us, bp_us);
    fclose(fp);
}

int tune_cached(Matrix &A, hipStream_t s, svr_tuning_t *out) {
    const char *path = getenv("SVR_TUNE_CACHE");
    if (!path || !*path) return tune(A, s, out);
    const std::string key = cache_key(A);
    int R = 0, T = 0;
    double uf = 0.0, ub = 0.0;
    if (cache_lookup(path, key, &R, &T, &uf, &ub)) {
        A.run_fwd = R;
        A.run_bp = T;
        if (out) {
            out->fwd_pairs_per_wave = R;
            out->bp_rows_per_group = T;
            out->fwd_pair_rows = A.pair_rows_eff();
            out->fwd_us = uf;
            out->bp_us = ub;
            out->fwd_natural_order = A.xcd_bands ? 0 : 1;
        }
        return SVR_OK;
    }
    svr_tuning_t t{};
    const int rc = tune(A, s, &t);
    if (rc) return rc;
    cache_store(path, key, t.fwd_pairs_per_wave, t.bp_rows_per_group, t.fwd_us, t.bp_us);
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
    return SVR_OK;
}

int svr_matrix_set_tuning(svr_matrix *A, const svr_tuning_t *t) {
    svr::clear_error();
    SVR_REQUIRE(A && t, "NULL argument");
    SVR_REQUIRE(t->fwd_pairs_per_wave >= 0 && t->fwd_pairs_per_wave <= 31, "fwd_pairs_per_wave must be in [0, 31]");
    SVR_REQUIRE(t->bp_rows_per_group >= 0 && t->bp_rows_per_group <= 1024, "bp_rows_per_group must be in [0, 1024]");
    SVR_REQUIRE(t->fwd_pair_rows >= 0, "fwd_pair_rows must be >= 0");
    SVR_REQUIRE(t->fwd_natural_order == 0 || t->fwd_natural_order == 1, "fwd_natural_order must be 0 or 1");
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
