// System-matrix builder: exact ray/pixel intersection lengths (Siddon's
// method) for the linear model E[g] = A f + w (Sec. 2.1, eq. voxel_td), laid
// out by ordered subsets (Sec. 2.1) for gather-only projectors.
//
// One thread traces one ray in FP64, pixel units, merging the crossings with
// the vertical and horizontal grid lines in increasing ray parameter and
// assigning each piece to the pixel that contains its midpoint.  This file is
// compiled without floating-point contraction so that every crossing,
// midpoint and length is the correctly rounded result of the operations as
// written (the pixel a piece falls in is an integer decision taken in FP64).
#include <algorithm>
#include <climits>
#include <cmath>

#include "common.h"
#include "util.h"

#pragma clang fp contract(off)

namespace svr {

constexpr double SEG_EPS = 1e-9;     // pieces shorter than this (pixel units) are dropped
constexpr double SNAP_EPS = 1e-12;   // |cos|,|sin| below this are snapped to 0

struct Ray {
    double ox, oy, dx, dy;
};

// Ray (v, b) in grid coordinates: origin u*(cos, sin) + (nx/2, ny/2), unit
// direction (-sin, cos), u = (b - (B-1)/2) * bin/pixel.
__device__ inline Ray make_ray(const svr_geometry &g, int v, int b) {
    double th = ((double)v * g.arc_rad) / (double)g.n_views;
    double c = cos(th), s = sin(th);
    if (fabs(c) < SNAP_EPS) { c = 0.0; s = copysign(1.0, s); }
    if (fabs(s) < SNAP_EPS) { s = 0.0; c = copysign(1.0, c); }
    double u = ((double)b - (double)(g.n_bins - 1) / 2.0) * (g.bin_mm / g.pixel_mm);
    Ray r;
    r.ox = u * c + (double)g.nx / 2.0;
    r.oy = u * s + (double)g.ny / 2.0;
    r.dx = -s;
    r.dy = c;
    return r;
}

// Visits the pieces of a ray in increasing parameter: emit(pixel, length_in_pixels).
template <class Emit>
__device__ inline void trace(const svr_geometry &g, const Ray &r, Emit &&emit) {
    const int nx = g.nx, ny = g.ny;
    int xi = 0, xs = 0, xleft = 0, yi = 0, ys = 0, yleft = 0;
    if (r.dx < 0.0) { xi = nx; xs = -1; xleft = nx + 1; }
    else if (r.dx > 0.0) { xi = 0; xs = 1; xleft = nx + 1; }
    if (r.dy < 0.0) { yi = ny; ys = -1; yleft = ny + 1; }
    else if (r.dy > 0.0) { yi = 0; ys = 1; yleft = ny + 1; }
    double tprev = 0.0;
    bool have = false;
    while (xleft > 0 || yleft > 0) {
        double tx = xleft > 0 ? ((double)xi - r.ox) / r.dx : INFINITY;
        double ty = yleft > 0 ? ((double)yi - r.oy) / r.dy : INFINITY;
        double t;
        if (tx <= ty) { t = tx; xi += xs; --xleft; }
        else { t = ty; yi += ys; --yleft; }
        if (have) {
            double seg = t - tprev;
            if (seg >= SEG_EPS) {
                double tm = (tprev + t) * 0.5;
                double X = r.ox + tm * r.dx;
                double Y = r.oy + tm * r.dy;
                double fx = floor(X), fy = floor(Y);
                if (fx >= 0.0 && fx < (double)nx && fy >= 0.0 && fy < (double)ny)
                    emit((int)fy * nx + (int)fx, seg);
            }
        }
        tprev = t;
        have = true;
    }
}

template <typename WT> __device__ inline WT store_w(double v);
template <> __device__ inline float store_w<float>(double v) { return (float)v; }
template <> __device__ inline _Float16 store_w<_Float16>(double v) { return (_Float16)(float)v; }
template <> __device__ inline bf16_t store_w<bf16_t>(double v) {
    // FP64 -> FP32 (nearest even) -> BF16 (nearest even); weights are finite.
    uint32_t u = __float_as_uint((float)v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    bf16_t r;
    r.bits = (uint16_t)(u >> 16);
    return r;
}

// subset-ordered row r -> natural sinogram index
__global__ void k_row_sino(int M, int B, int Ns, const int *row_start, int *row_sino) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= M) return;
    int lo = 0, hi = Ns;  // find t with row_start[t] <= r < row_start[t+1]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (row_start[mid] <= r) lo = mid; else hi = mid;
    }
    int t = lo;
    int local = r - row_start[t];
    int j = local / B, b = local - j * B;
    int v = t + j * Ns;
    row_sino[r] = v * B + b;
}

__global__ void k_siddon_count(svr_geometry g, int M, const int *row_sino, int *counts) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= M) return;
    int m = row_sino[r];
    int v = m / g.n_bins, b = m - v * g.n_bins;
    Ray ray = make_ray(g, v, b);
    int c = 0;
    trace(g, ray, [&](int, double) { ++c; });
    counts[r] = c;
}

template <typename WT, typename IT>
__global__ void k_siddon_fill(svr_geometry g, int M, const int *row_sino, const int *row_ptr,
                              const float *mu, IT *col, WT *val) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= M) return;
    int m = row_sino[r];
    int v = m / g.n_bins, b = m - v * g.n_bins;
    Ray ray = make_ray(g, v, b);
    const double pmm = g.pixel_mm;
    double att = 1.0;
    if (mu) {
        double lineint = 0.0;
        trace(g, ray, [&](int pix, double seg) { lineint = lineint + (seg * pmm) * (double)mu[pix]; });
        att = exp(-lineint);
    }
    int pos = row_ptr[r];
    trace(g, ray, [&](int pix, double seg) {
        double len = seg * pmm;
        if (mu) len = len * att;
        col[pos] = (IT)pix;
        val[pos] = store_w<WT>(len);
        ++pos;
    });
}

// ---- transposition (per subset), deterministic ------------------------------
// Entries per (subset, pixel), and each entry's arrival rank among its
// transposed row's entries (slot, any order).  A subset's rows, hence its
// entries, are one contiguous range of A, so a workgroup per (subset, chunk of
// CC_PIX pixels) reads that range once, counts the entries of its chunk in an
// LDS histogram (the atomic's return value is the slot) and writes the
// chunk's counts: no global atomics, and every count is written once, so the
// counts need no clearing.
constexpr int CC_PIX = 16384;  // 64 KB of int counts per workgroup
constexpr int CC_THREADS = 1024;
#ifndef SVR_CC_ILP
#define SVR_CC_ILP 16
#endif
constexpr int CC_ILP = SVR_CC_ILP;
template <typename IT>
__global__ void __launch_bounds__(CC_THREADS)
k_col_count(int N, int chunks, const int *row_start, const int *row_ptr, const IT *col, int *cnt, int *slot) {
    __shared__ int hist[CC_PIX];
    const int t = (int)blockIdx.x / chunks, c = (int)blockIdx.x - t * chunks;
    const int n0 = c * CC_PIX, n1 = min(N, n0 + CC_PIX);
    for (int k = threadIdx.x; k < CC_PIX; k += CC_THREADS) hist[k] = 0;
    __syncthreads();
    const int i0 = row_ptr[row_start[t]], i1 = row_ptr[row_start[t + 1]];
    // CC_ILP entries a thread per pass, all loaded before any is used, so that
    // the pass waits on one memory latency, not CC_ILP of them
    for (int base = i0 + (int)threadIdx.x; base < i1; base += CC_THREADS * CC_ILP) {
        int n[CC_ILP];
#pragma unroll
        for (int k = 0; k < CC_ILP; ++k) {
            const int i = base + k * CC_THREADS;
            n[k] = i < i1 ? (int)col[i] : -1;
        }
#pragma unroll
        for (int k = 0; k < CC_ILP; ++k)
            if (n[k] >= n0 && n[k] < n1) slot[base + k * CC_THREADS] = atomicAdd(&hist[n[k] - n0], 1);
    }
    __syncthreads();
    int *out = cnt + (int64_t)t * N;
    for (int n = n0 + (int)threadIdx.x; n < n1; n += CC_THREADS) out[n] = hist[n - n0];
}

// A transposed entry between the fill and the ranking: its subset-local row
// in the low 32 bits, its weight's bits in the high ones, so that the fill's
// scattered writes are one 8-byte store per entry
template <typename WT>
__device__ inline uint64_t pack_entry(int row, WT v) {
    uint32_t bits;
    if constexpr (sizeof(WT) == 4) bits = __builtin_bit_cast(uint32_t, v);
    else bits = (uint32_t)__builtin_bit_cast(uint16_t, v);
    return (uint64_t)(uint32_t)row | ((uint64_t)bits << 32);
}
__device__ inline int entry_row(uint64_t e) { return (int)(uint32_t)e; }
template <typename WT>
__device__ inline WT entry_val(uint64_t e) {
    const uint32_t bits = (uint32_t)(e >> 32);
    if constexpr (sizeof(WT) == 4) return __builtin_bit_cast(WT, bits);
    else return __builtin_bit_cast(WT, (uint16_t)bits);
}

// every entry of A into its transposed row at the slot k_col_count gave it
// (k_rank_T orders each row afterwards); a wavefront per row of A, lanes over
// its entries
template <typename WT, typename IT>
__global__ void k_fill_T(int M, int B, int Ns, int N, const int *row_sino, const int *row_start,
                         const int *row_ptr, const IT *col, const WT *val, const int *ptrT,
                         const int *slot, uint64_t *fill) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = (int)(gid >> 6), lane = (int)(gid & 63);
    if (r >= M) return;
    const int t = (row_sino[r] / B) % Ns;
    const int local = r - row_start[t];
    const int64_t base = (int64_t)t * N;
    for (int i = row_ptr[r] + lane; i < row_ptr[r + 1]; i += 64) {
        fill[ptrT[base + col[i]] + slot[i]] = pack_entry(local, val[i]);
    }
}

// Each transposed row in subset-local row order (view, then bin), read from
// the unordered fill (keys, vals) and written to (rowT, valT): a 32-lane group
// per R consecutive rows, two groups per wavefront; the lane holding an entry
// counts the keys of its row that are smaller (every key broadcast lane by
// lane) and writes the entry at beg + that rank.  Keys of a row are unique, so
// the ranks are a permutation and the order is the ascending one, whatever
// order the fill left.  The group loads its R rows' bounds and first 32
// entries before ranking any of them, so that R rows' loads are in flight at
// once (the kernel waits on memory, not on its compares); a row longer than 32
// (in either group of the wavefront) is ranked from memory in 32-entry chunks.
// Every lane of a wavefront runs the loops (their bounds are the longer of the
// wavefront's two rows).
#ifndef SVR_RANK_ROWS
#define SVR_RANK_ROWS 4
#endif
constexpr int RANK_ROWS = SVR_RANK_ROWS;
template <typename WT, typename IT, int R>
__global__ void __launch_bounds__(256)
k_rank_T(int64_t nrows, const int *ptrT, const uint64_t *fill, IT *rowT, WT *valT) {
    const int lane = threadIdx.x & 63, h = lane >> 5, gl = lane & 31;
    const int64_t q0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 5) * R;
    const int pv = (gl <= R && q0 + gl <= nrows) ? ptrT[q0 + gl] : 0;  // row bounds, one per lane
    int beg[R], len[R], key[R];
    WT val[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int b = __shfl(pv, (h << 5) + r), e = __shfl(pv, (h << 5) + r + 1);
        const bool has_row = q0 + r < nrows;
        beg[r] = has_row ? b : 0;
        len[r] = has_row ? e - b : 0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool has = gl < len[r];
        const uint64_t ent = has ? fill[beg[r] + gl] : 0;
        key[r] = has ? entry_row(ent) : INT_MAX;
        val[r] = entry_val<WT>(ent);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int lmax = max(__builtin_amdgcn_readlane(len[r], 0), __builtin_amdgcn_readlane(len[r], 32));
        if (lmax <= 32) {
            int rank = 0;
#pragma unroll 4
            for (int j = 0; j < lmax; ++j) {
                const int k0 = __builtin_amdgcn_readlane(key[r], j), k1 = __builtin_amdgcn_readlane(key[r], 32 + j);
                rank += (h ? k1 : k0) < key[r];
            }
            if (gl < len[r]) {
                rowT[beg[r] + rank] = (IT)key[r];
                valT[beg[r] + rank] = val[r];
            }
            continue;
        }
        for (int c = 0; c < lmax; c += 32) {
            const int e = c + gl;
            const bool has = e < len[r];
            const uint64_t ent = has ? fill[beg[r] + e] : 0;
            const int k = has ? entry_row(ent) : INT_MAX;
            int rank = 0;
            for (int d = 0; d < lmax; d += 32) {
                const int kd = d + gl < len[r] ? entry_row(fill[beg[r] + d + gl]) : INT_MAX;
#pragma unroll 8
                for (int j = 0; j < 32; ++j) {
                    const int k0 = __builtin_amdgcn_readlane(kd, j), k1 = __builtin_amdgcn_readlane(kd, 32 + j);
                    rank += (h ? k1 : k0) < k;
                }
            }
            if (has) {
                rowT[beg[r] + rank] = (IT)k;
                valT[beg[r] + rank] = entry_val<WT>(ent);
            }
        }
    }
}

// sens_t = A_t^T 1 (FP64 sum in transposed-row order, stored FP32), sens = sum_t (FP64)
template <typename WT>
__global__ void k_sens(int Ns, int N, const int *ptrT, const WT *valT, float *sens_t, double *sens) {
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double tot = 0.0;
    for (int t = 0; t < Ns; ++t) {
        int64_t q = (int64_t)t * N + n;
        double s = 0.0;
        const int e = ptrT[q + 1];
        // eight loads in flight, summed in entry order (valT's zero padding past its last
        // non-zero keeps the loads past e in bounds)
        for (int i = ptrT[q]; i < e; i += 8) {
            WT v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = valT[i + k];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (i + k < e) s = s + (double)load_w(v[k]);
        }
        sens_t[q] = (float)s;
        tot = tot + s;
    }
    sens[n] = tot;
}

// stats[0] = longest row, stats[1] = longest transposed row, stats[2 + t] =
// row_ptr at the first row of subset t (t = 0..Ns)
// Maxima: a grid-stride loop, a block reduction and one integer atomic per
// block.  Atomics on one address serialise (an atomic per element or per
// wavefront took 245 us for the 1.4 M transposed row counts at 256^2), so
// these kernels run at most MAX_BLOCKS blocks.
constexpr int MAX_BLOCKS = 256;
__device__ inline void block_max_to(int v, int *dst) {
    __shared__ int red[256 / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = red[0];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) m = max(m, red[k]);
        atomicMax(dst, m);
    }
}
__global__ void __launch_bounds__(256) k_row_stats(int M, const int *row_ptr, int *stats) {
    int v = 0;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < M; r += gridDim.x * blockDim.x)
        v = max(v, row_ptr[r + 1] - row_ptr[r]);
    block_max_to(v, &stats[0]);
}
__global__ void __launch_bounds__(256) k_max_count(int64_t n, const int *cnt, int *stats) {
    int v = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v = max(v, cnt[i]);
    block_max_to(v, &stats[1]);
}
__global__ void k_subset_offsets(int Ns, const int *row_start, const int *row_ptr, int *stats) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t <= Ns) stats[2 + t] = row_ptr[row_start[t]];
}

// forward indices in tiled pixel order; the pad entries stay 0
// (8 bytes of indices a thread: one load and one store)
template <typename IT>
constexpr int TILE_COLS_V = 8 / (int)sizeof(IT);
template <typename IT>
__global__ void k_tile_cols(const IT *col, int64_t n_all, int64_t nnz, int nx, int tx, IT *colt) {
    constexpr int V = TILE_COLS_V<IT>;
    struct alignas(8) Pack {
        IT v[V];
    };
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * V;
    if (i0 >= n_all) return;
    if (i0 + V <= n_all) {  // the arrays' bases are 256-byte aligned, i0 a multiple of V
        Pack p = *(const Pack *)(col + i0);
#pragma unroll
        for (int k = 0; k < V; ++k) p.v[k] = i0 + k < nnz ? (IT)tiled_index((int)p.v[k], nx, tx) : (IT)0;
        *(Pack *)(colt + i0) = p;
    } else {
        for (int64_t i = i0; i < n_all; ++i) colt[i] = i < nnz ? (IT)tiled_index((int)col[i], nx, tx) : (IT)0;
    }
}

// Every slot p of the tiled copy: the pixel it holds (the inverse of
// tiled_index_xy), or 0 for the slots of partial tiles outside the image, so
// the copy needs no clearing first; the writes are coalesced.
__global__ void k_tile_image(const float *f, int nx, int ny, int tx, int Nt, float *ft) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= Nt) return;
    const int tile = p / (TILE_W * TILE_H), w = p - tile * (TILE_W * TILE_H);
    const int ty = tile / tx, tc = tile - ty * tx;
    const int iy = ty * TILE_H + w / TILE_W, ix = tc * TILE_W + w % TILE_W;
    ft[p] = (ix < nx && iy < ny) ? f[iy * nx + ix] : 0.0f;
}

int launch_tile_image(const Matrix &A, const float *f, float *ft, hipStream_t s) {
    k_tile_image<<<(A.Nt + 255) / 256, 256, 0, s>>>(f, A.geom.nx, A.geom.ny, A.tx, A.Nt, ft);
    SVR_HIP(hipGetLastError());
    return SVR_OK;
}

// The build, with its index arrays (col, rowT and the tiled copy of col) of
// type IT from the start: uint16 when every pixel index and every subset-local
// row fits in 16 bits (the geometry fixes both before any ray is traced)
template <typename WT, typename IT>
static int build_indexed(Matrix &A, const float *mu, hipStream_t s) {
    const int M = A.M, N = A.N, Ns = A.Ns, B = A.geom.n_bins;
    const int T = 256;
    const int gM = (M + T - 1) / T;
    const int64_t NT = (int64_t)Ns * N;
    struct Temps {  // the build's temporaries, freed (stream-ordered) on every return
        int *counts = nullptr, *cnt = nullptr, *stats = nullptr, *slot = nullptr;
        uint64_t *fill = nullptr;
        ~Temps() {
            dfree(counts);
            dfree(cnt);
            dfree(stats);
            dfree(slot);
            dfree(fill);
        }
    } tmp;
    int *&counts = tmp.counts, *&cnt = tmp.cnt, *&stats = tmp.stats;
    SVR_HIP(dalloc(&counts, M));
    SVR_HIP(dalloc(&stats, Ns + 3));
    SVR_HIP(hipMemsetAsync(stats, 0, sizeof(int) * (Ns + 3), s));
    k_siddon_count<<<gM, T, 0, s>>>(A.geom, M, A.d_row_sino, counts);
    SVR_HIP(hipGetLastError());
    SVR_HIP(dalloc(&A.d_row_ptr, M + 1));
    int64_t nnz = 0;
    int rc = exclusive_scan(counts, M, A.d_row_ptr, &nnz, s);  // synchronises: nnz sizes the arrays
    if (rc) return rc;
    A.nnz = nnz;
    WT *val = nullptr, *valT = nullptr;
    IT *col = nullptr, *rowT = nullptr, *colt = nullptr;
    SVR_HIP(dalloc(&col, nnz + NNZ_PAD));
    SVR_HIP(dalloc(&val, nnz + NNZ_PAD));
    SVR_HIP(dalloc(&rowT, nnz + NNZ_PAD));
    SVR_HIP(dalloc(&valT, nnz + NNZ_PAD));
    SVR_HIP(hipMemsetAsync(col + nnz, 0, sizeof(IT) * NNZ_PAD, s));
    SVR_HIP(hipMemsetAsync(val + nnz, 0, sizeof(WT) * NNZ_PAD, s));
    SVR_HIP(hipMemsetAsync(rowT + nnz, 0, sizeof(IT) * NNZ_PAD, s));
    SVR_HIP(hipMemsetAsync(valT + nnz, 0, sizeof(WT) * NNZ_PAD, s));
    A.d_col = col;
    A.d_rowT = rowT;
    SVR_HIP(dalloc(&cnt, NT));
    SVR_HIP(dalloc(&A.d_ptrT, NT + 1));
    SVR_HIP(dalloc(&A.d_sens_t, NT));
    SVR_HIP(dalloc(&A.d_sens, N));
    A.d_val = val;
    A.d_valT = valT;
    k_siddon_fill<WT, IT><<<gM, T, 0, s>>>(A.geom, M, A.d_row_sino, A.d_row_ptr, mu, col, val);
    k_row_stats<<<std::min<unsigned>(gM, MAX_BLOCKS), T, 0, s>>>(M, A.d_row_ptr, stats);
    k_subset_offsets<<<(Ns + 1 + T - 1) / T, T, 0, s>>>(Ns, A.d_row_start, A.d_row_ptr, stats);
    // transposed rows per subset
    const unsigned gW = (unsigned)(((int64_t)M * 64 + T - 1) / T);  // a wavefront per row
    // each entry's slot: in rowT when that holds int32 (k_rank_T writes rowT
    // after the last read of the slots), else in a buffer of its own
    int *slot = nullptr;
    if constexpr (sizeof(IT) == sizeof(int)) {
        slot = (int *)rowT;
    } else {
        SVR_HIP(dalloc(&tmp.slot, nnz));
        slot = tmp.slot;
    }
    const int chunks = (N + CC_PIX - 1) / CC_PIX;
    k_col_count<IT><<<(unsigned)((int64_t)Ns * chunks), CC_THREADS, 0, s>>>(N, chunks, A.d_row_start, A.d_row_ptr,
                                                                         col, cnt, slot);
    k_max_count<<<(unsigned)std::min<int64_t>((NT + T - 1) / T, MAX_BLOCKS), T, 0, s>>>(NT, cnt, stats);
    SVR_HIP(hipGetLastError());
    int64_t nnzT = 0;
    rc = exclusive_scan(cnt, NT, A.d_ptrT, &nnzT, s);
    if (rc) return rc;
    if (nnzT != nnz) { set_error("transpose count mismatch"); return SVR_EDEVICE; }
    SVR_HIP(dalloc(&tmp.fill, nnz));
    k_fill_T<WT, IT><<<gW, T, 0, s>>>(M, B, Ns, N, A.d_row_sino, A.d_row_start, A.d_row_ptr, col,
                                      val, A.d_ptrT, slot, tmp.fill);
    const int64_t groups = (NT + RANK_ROWS - 1) / RANK_ROWS;
    k_rank_T<WT, IT, RANK_ROWS><<<(unsigned)((groups * 32 + T - 1) / T), T, 0, s>>>(NT, A.d_ptrT, tmp.fill,
                                                                                   rowT, valT);
    dfree(tmp.fill);  // stream-ordered: after the ranking
    tmp.fill = nullptr;
    k_sens<WT><<<(N + T - 1) / T, T, 0, s>>>(Ns, N, A.d_ptrT, valT, A.d_sens_t, A.d_sens);
    // the forward indices in tiled pixel order
    SVR_HIP(dalloc(&colt, nnz + NNZ_PAD));
    const int64_t packs = (nnz + NNZ_PAD + TILE_COLS_V<IT> - 1) / TILE_COLS_V<IT>;
    k_tile_cols<IT><<<(unsigned)((packs + T - 1) / T), T, 0, s>>>(col, nnz + NNZ_PAD, nnz, A.geom.nx, A.tx, colt);
    A.d_colt = colt;
    SVR_HIP(hipGetLastError());
    std::vector<int> h(Ns + 3);
    SVR_HIP(hipMemcpyAsync(h.data(), stats, sizeof(int) * (Ns + 3), hipMemcpyDeviceToHost, s));
    SVR_HIP(hipStreamSynchronize(s));
    A.max_row_nnz = h[0];
    A.max_col_nnz = h[1];
    A.nnz_sub.assign(Ns, 0);
    for (int t = 0; t < Ns; ++t) A.nnz_sub[t] = (int64_t)h[2 + t + 1] - h[2 + t];
    A.bytes = (int64_t)sizeof(int) * (2 * (M + 1) + NT + 1 + (Ns + 1)) + (int64_t)sizeof(IT) * 3 * (nnz + NNZ_PAD) +
              (int64_t)A.wbytes() * 2 * (nnz + NNZ_PAD) + (int64_t)sizeof(float) * NT + (int64_t)sizeof(double) * N;
    return SVR_OK;
}

template <typename WT>
static int build_typed(Matrix &A, const float *mu, hipStream_t s) {
    int max_rows = 0;
    for (int t = 0; t < A.Ns; ++t) max_rows = std::max(max_rows, A.rows_of(t));
    A.tx = tiles_x(A.geom.nx);
    A.Nt = tiled_count(A.geom.nx, A.geom.ny);
    A.idx16 = A.idx16 && A.Nt <= 65536 && max_rows <= 65536;
    return A.idx16 ? build_indexed<WT, uint16_t>(A, mu, s) : build_indexed<WT, int>(A, mu, s);
}

int build_matrix(Matrix &A, const float *mu_dev, hipStream_t s) {
    AllocStream as(s);
    A.owner = s;
    const svr_geometry &g = A.geom;
    const int Ns = A.Ns, B = g.n_bins;
    A.M = g.n_views * B;
    A.N = g.nx * g.ny;
    A.row_start.assign(Ns + 1, 0);
    for (int t = 0; t < Ns; ++t) {
        int nv = (g.n_views - t + Ns - 1) / Ns;  // views t, t+Ns, ... below n_views
        A.row_start[t + 1] = A.row_start[t] + nv * B;
    }
    SVR_HIP(dalloc(&A.d_row_start, Ns + 1));
    SVR_HIP(hipMemcpyAsync(A.d_row_start, A.row_start.data(), sizeof(int) * (Ns + 1),
                           hipMemcpyHostToDevice, s));
    SVR_HIP(dalloc(&A.d_row_sino, A.M));
    k_row_sino<<<(A.M + 255) / 256, 256, 0, s>>>(A.M, B, Ns, A.d_row_start, A.d_row_sino);
    SVR_HIP(hipGetLastError());
    switch (A.wtype) {
        case SVR_W_F32: return build_typed<float>(A, mu_dev, s);
        case SVR_W_F16: return build_typed<_Float16>(A, mu_dev, s);
        case SVR_W_BF16: return build_typed<bf16_t>(A, mu_dev, s);
    }
    set_error("unknown weight type %d", A.wtype);
    return SVR_EINVAL;
}

}  // namespace svr
