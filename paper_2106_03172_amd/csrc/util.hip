// Small device utilities: exclusive scan, deterministic FP64 reduction,
// row permutation, input validation counters.
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cmath>

#include "common.h"
#include "kernels.h"
#include "util.h"

namespace svr {

// ---------------------------------------------------------------------------
// errors and allocation
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
}
void clear_error() { g_err.clear(); }
const char *last_error() { return g_err.c_str(); }

LaunchEvents &pending_timing() {
    static thread_local LaunchEvents t;
    return t;
}

static std::atomic<long> g_alloc_budget{-2};  // -2: not read yet, -1: unlimited
static thread_local hipStream_t g_alloc_stream = nullptr;
static thread_local BlockCache *g_cache = nullptr;
static thread_local bool g_cache_keep = false;

AllocStream::AllocStream(hipStream_t s) : prev(g_alloc_stream) { g_alloc_stream = s; }
AllocStream::~AllocStream() { g_alloc_stream = prev; }

BlockCacheScope::BlockCacheScope(BlockCache *c, bool keep) : prev_cache(g_cache), prev_keep(g_cache_keep) {
    g_cache = c;
    g_cache_keep = keep;
}
BlockCacheScope::~BlockCacheScope() {
    g_cache = prev_cache;
    g_cache_keep = prev_keep;
}

void block_cache_trim(BlockCache &c, int64_t max_idle) {
    std::lock_guard<std::mutex> lk(c.mu);
    while (c.idle_bytes > max_idle && !c.idle.empty()) {
        auto it = std::prev(c.idle.end());
        (void)hipFreeAsync(it->second, g_alloc_stream);
        c.idle_bytes -= (int64_t)it->first;
        c.idle.erase(it);
    }
}

// keep freed blocks in the device's default pool instead of returning them
// to the driver at every synchronisation
static void keep_pool_memory() {
    static thread_local int done_dev = -1;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev == done_dev) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t big = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &big);
    }
    done_dev = dev;
}

hipError_t dmalloc(void **p, size_t bytes) {
    long b = g_alloc_budget.load();
    if (b == -2) {
        const char *e = getenv("SVR_FAULT_ALLOC_AFTER");
        g_alloc_budget.compare_exchange_strong(b, e ? atol(e) : -1);
        b = g_alloc_budget.load();
    }
    while (b > 0 && !g_alloc_budget.compare_exchange_weak(b, b - 1)) {
    }
    if (b == 0) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    if (bytes == 0) bytes = 16;
    BlockCache *c = g_cache;
    if (c) {
        std::lock_guard<std::mutex> lk(c->mu);
        auto it = c->idle.lower_bound(bytes);
        if (it != c->idle.end() && it->first <= bytes + bytes / 4) {
            *p = it->second;
            c->out[it->second] = it->first;
            c->idle_bytes -= (int64_t)it->first;
            c->idle.erase(it);
            ++c->reuses;
            return hipSuccess;
        }
    }
    keep_pool_memory();
    const hipError_t e = hipMallocAsync(p, bytes, g_alloc_stream);
    if (c && e == hipSuccess) {
        // assigned, not inserted: an entry left by a block the cache handed out but that was
        // freed outside its scope may name the same address with another size
        std::lock_guard<std::mutex> lk(c->mu);
        c->out[*p] = bytes;
    }
    return e;
}

void dfree(void *p) {
    if (!p) return;
    if (BlockCache *c = g_cache) {
        std::lock_guard<std::mutex> lk(c->mu);
        auto it = c->out.find(p);
        if (it != c->out.end()) {
            if (g_cache_keep) {
                c->idle.emplace(it->second, p);
                c->idle_bytes += (int64_t)it->second;
                c->out.erase(it);
                return;
            }
            c->out.erase(it);
        }
    }
    (void)hipFreeAsync(p, g_alloc_stream);
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 counts: out[0..n] (out[n] = total), int64 total
// ---------------------------------------------------------------------------
constexpr int SCAN_T = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_CHUNK = SCAN_T * SCAN_ITEMS;

__global__ void __launch_bounds__(SCAN_T) k_scan_blocksum(const int *in, int64_t n, int64_t *bsum) {
    __shared__ int64_t red[SCAN_T];
    int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t s = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (base + i < n) s += in[base + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = SCAN_T / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

// single block: exclusive scan of nb block sums in place; total to bsum[nb]
__global__ void __launch_bounds__(1024) k_scan_blocksums(int64_t *bsum, int nb) {
    __shared__ int64_t part[1024];
    int per = (nb + 1023) / 1024;
    int beg = threadIdx.x * per;
    int64_t s = 0;
    for (int i = 0; i < per; ++i)
        if (beg + i < nb) s += bsum[beg + i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int i = 0; i < 1024; ++i) {
            int64_t v = part[i];
            part[i] = run;
            run += v;
        }
        bsum[nb] = run;
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int i = 0; i < per; ++i)
        if (beg + i < nb) {
            int64_t v = bsum[beg + i];
            bsum[beg + i] = run;
            run += v;
        }
}

__global__ void __launch_bounds__(SCAN_T) k_scan_apply(const int *in, int64_t n, const int64_t *bsum, int *out) {
    __shared__ int64_t pre[SCAN_T];
    int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t s = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (base + i < n) s += in[base + i];
    pre[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of thread sums
    for (int w = 1; w < SCAN_T; w <<= 1) {
        int64_t add = ((int)threadIdx.x >= w) ? pre[threadIdx.x - w] : 0;
        __syncthreads();
        pre[threadIdx.x] += add;
        __syncthreads();
    }
    int64_t run = bsum[blockIdx.x] + pre[threadIdx.x] - s;
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (base + i < n) {
            out[base + i] = (int)run;
            run += in[base + i];
        }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_T - 1) out[n] = (int)bsum[gridDim.x];
}

int exclusive_scan(const int *in, int64_t n, int *out, int64_t *total, hipStream_t s) {
    AllocStream as(s);
    int nb = (int)((n + SCAN_CHUNK - 1) / SCAN_CHUNK);
    if (nb < 1) nb = 1;
    int64_t *bsum = nullptr;
    SVR_HIP(dalloc(&bsum, nb + 1));
    k_scan_blocksum<<<nb, SCAN_T, 0, s>>>(in, n, bsum);
    k_scan_blocksums<<<1, 1024, 0, s>>>(bsum, nb);
    SVR_HIP(hipMemcpyAsync(total, bsum + nb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SVR_HIP(hipStreamSynchronize(s));
    // headroom below INT32_MAX: the kernels that walk a range of these offsets step an int
    // index up to a few workgroups past its end
    if (*total < 0 || *total > INT32_MAX - 65536) {
        dfree(bsum);
        set_error("scan total %lld exceeds the int32 index range", (long long)*total);
        return SVR_EINVAL;
    }
    k_scan_apply<<<nb, SCAN_T, 0, s>>>(in, n, bsum, out);
    SVR_HIP(hipGetLastError());
    dfree(bsum);  // stream-ordered: after k_scan_apply
    return SVR_OK;
}

// ---------------------------------------------------------------------------
// deterministic FP64 sum: one block, fixed strided order then a fixed tree
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_reduce_sum(const double *part, int n, double *out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

int launch_reduce_sum(const double *part, int n, double *out, hipStream_t s) {
    k_reduce_sum<<<1, 256, 0, s>>>(part, n, out);
    SVR_HIP(hipGetLastError());
    return SVR_OK;
}

// ---------------------------------------------------------------------------
// sinogram permutation natural -> subset order
// ---------------------------------------------------------------------------
__global__ void k_gather_rows(const int *row_sino, int M, const float *src, float *dst) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < M) dst[r] = src[row_sino[r]];
}

int launch_gather_rows(const Matrix &A, const float *src_nat, float *dst_sub, hipStream_t s) {
    k_gather_rows<<<(A.M + 255) / 256, 256, 0, s>>>(A.d_row_sino, A.M, src_nat, dst_sub);
    SVR_HIP(hipGetLastError());
    return SVR_OK;
}

// ---------------------------------------------------------------------------
// validation: count entries that are non-finite, negative, or (if
// require_positive) not strictly positive
// ---------------------------------------------------------------------------
__global__ void k_count_bad(const float *x, int64_t n, int require_positive, int *counter) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    if (i < n) {
        float v = x[i];
        bad = !isfinite(v) || v < 0.0f || (require_positive && !(v > 0.0f));
    }
    // wave vote then one atomic per wave (integer atomics only)
    unsigned long long m = __ballot(bad);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(counter, __popcll(m));
}

int launch_count_bad(const float *x, int64_t n, int require_positive, int *counter, hipStream_t s) {
    if (n <= 0) return SVR_OK;
    k_count_bad<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, n, require_positive, counter);
    SVR_HIP(hipGetLastError());
    return SVR_OK;
}

}  // namespace svr
