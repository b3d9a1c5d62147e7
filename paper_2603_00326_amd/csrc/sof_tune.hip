// sof_tune.hip -- crossover microbenchmark behind sof_autotune (paper section
// 4.1: histograms win on large nodes and sorting on small ones, and the
// crossover is measured once before training).
//
// For a ladder of node sizes s (2 .. 8192), a frontier of equal nodes of s
// contiguous rows (2^16 samples in all, k projections of nnz features; the
// rows are synthetic, or the caller's own with sof_autotune_on) is searched
// through sof_find_splits with all nodes on the sort path (T = INT32_MAX) and
// all on the histogram path (T = 0).  The chosen T is the smallest measured
// size from which the histogram path is never slower; sorting only loses
// ground as nodes grow (n log n against n), so once histograms have won at two
// consecutive sizes the larger sizes are not sorted.  The same frontiers
// searched with half the bins (sizes up to 1024) give the bin-count switch for
// small nodes: below the first size where full bins cost at most 10% more
// than half bins, nodes use half the bins.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <vector>

#include "sof.h"
#include "sof_host.h"

namespace sof {

__device__ __forceinline__ uint32_t tune_hash(uint32_t x) {
    // 32-bit integer finaliser of MurmurHash3 (Appleby)
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}

// X[f][r] uniform in [-1, 1) on a 2^-10 grid, labels hash % C
__global__ void k_tune_data(float* x, _Float16* xh, int32_t* y, int n_rows, int d, int C) {
    const int64_t total = (int64_t)n_rows * d;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t h = tune_hash((uint32_t)i * 2654435761u + 12345u);
        const float v = (float)((int)(h & 2047u) - 1024) * (1.0f / 1024.0f);
        x[i] = v;
        xh[i] = (_Float16)v;
        if (i < n_rows) y[i] = (int32_t)(tune_hash((uint32_t)i + 777u) % (uint32_t)C);
    }
}

// frontier of N nodes of s contiguous rows (row i mod n_rows for sample i);
// k projections per node, nnz distinct features each (consecutive from a
// hashed start), signs hashed
__global__ void k_tune_frontier(int32_t* node_off, int32_t* idx, int32_t* proj_off, int32_t* nz_off,
                                int32_t* nz_f, int8_t* nz_w, int N, int s, int k, int nnz, int d, int n_rows) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t v = t0; v <= N; v += stride) {
        node_off[v] = (int32_t)(v * s);
        proj_off[v] = (int32_t)(v * k);
    }
    for (int64_t i = t0; i < (int64_t)N * s; i += stride) idx[i] = (int32_t)(i % n_rows);
    const int64_t P = (int64_t)N * k;
    for (int64_t q = t0; q <= P; q += stride) nz_off[q] = (int32_t)(q * nnz);
    for (int64_t q = t0; q < P; q += stride) {
        const uint32_t h = tune_hash((uint32_t)q * 0x9e3779b9u + 99u);
        const int f0 = (int)(h % (uint32_t)(d - nnz + 1));
        for (int j = 0; j < nnz; ++j) {
            nz_f[q * nnz + j] = f0 + j;
            nz_w[q * nnz + j] = ((h >> (8 + j)) & 1u) ? (int8_t)-1 : (int8_t)1;
        }
    }
}

}  // namespace sof

using namespace sof;

namespace {

struct TuneBufs {
    std::vector<void*> ptrs;
    ~TuneBufs() {
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <class T>
    hipError_t get(T** p, size_t n) {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, n * sizeof(T) < 256 ? 256 : n * sizeof(T));
        if (e == hipSuccess) ptrs.push_back(q);
        *p = (T*)q;
        return e;
    }
};

}  // namespace

static int autotune_impl(sof_ctx* ctx, const sof_data* user, int32_t dtype, int32_t n_classes, int32_t k,
                         int32_t nnz, int32_t bins, sof_tune* out, void* stream) {
    if (!ctx || !out) return fail(SOF_ERR_INVALID_ARG, "sof_autotune: NULL argument");
    if (dtype != SOF_F32 && dtype != SOF_F16) return fail(SOF_ERR_UNSUPPORTED, "sof_autotune: dtype %d", dtype);
    if (n_classes < 2 || n_classes > SOF_MAX_CLASSES)
        return fail(SOF_ERR_UNSUPPORTED, "sof_autotune: n_classes %d", n_classes);
    if (k < 1 || k > 1024) return fail(SOF_ERR_INVALID_ARG, "sof_autotune: k %d outside [1, 1024]", k);
    if (nnz < 1 || nnz > SOF_MAX_NNZ) return fail(SOF_ERR_INVALID_ARG, "sof_autotune: nnz %d", nnz);
    if (bins < SOF_MIN_BINS || bins > SOF_MAX_BINS) return fail(SOF_ERR_UNSUPPORTED, "sof_autotune: bins %d", bins);
    if (user && user->n_features < nnz)
        return fail(SOF_ERR_INVALID_ARG, "sof_autotune_on: %d features, fewer than nnz %d", user->n_features, nnz);
    auto wall0 = std::chrono::steady_clock::now();
    memset(out, 0, sizeof(*out));
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");

    static const int kSizes[] = {2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024,
                                 1536, 2048, 3072, 4096, 6144, 8192};
    const int n_sizes = (int)(sizeof(kSizes) / sizeof(kSizes[0]));
    static_assert(sizeof(kSizes) / sizeof(kSizes[0]) <= 32, "sof_tune holds 32 points");
    // the caller's rows (at most 2^16 of them, its first 64 features) or 2^16
    // synthetic rows
    const int n_rows = user ? (user->n_rows < (1 << 16) ? user->n_rows : (1 << 16)) : (1 << 16);
    const int d = user ? (user->n_features < 64 ? user->n_features : 64) : 64;
    const int kk = k > 64 ? 64 : k;   // per node-projection cost is what is compared
    int maxN = 0;
    for (int i = 0; i < n_sizes; ++i) maxN = n_rows / kSizes[i] > maxN ? n_rows / kSizes[i] : maxN;
    // The two wave tiles are compared on frontiers that fill the GPU (4
    // nodes per compute unit; rows repeat): with only 2^16 rows the larger
    // sizes have too few nodes for the wave-per-projection tile's one block
    // per node, and the block tile would win for that reason alone.
    const int n_tile = 4 * ctx->n_cu;
    if (n_tile > maxN) maxN = n_tile;
    const int64_t maxP = (int64_t)maxN * kk;
    const int64_t max_idx = (int64_t)n_tile * kMidSplit > n_rows ? (int64_t)n_tile * kMidSplit : n_rows;

    TuneBufs B;
    float* x = nullptr;
    _Float16* xh = nullptr;
    int32_t *y = nullptr, *no, *idx, *po, *zo, *zf, *node_bins;
    int8_t* zw;
    sof_split* sp;
    if ((!user && ((e = B.get(&x, (size_t)n_rows * d)) || (e = B.get(&xh, (size_t)n_rows * d)) ||
                   (e = B.get(&y, n_rows)))) ||
        (e = B.get(&no, maxN + 1)) || (e = B.get(&idx, (size_t)max_idx)) || (e = B.get(&po, maxN + 1)) ||
        (e = B.get(&zo, maxP + 1)) || (e = B.get(&zf, maxP * nnz)) || (e = B.get(&zw, maxP * nnz)) ||
        (e = B.get(&sp, maxN)) || (e = B.get(&node_bins, maxN)))
        return hip_fail(e, "sof_autotune: hipMalloc");
    if (!user) hipLaunchKernelGGL(k_tune_data, dim3(1024), dim3(256), 0, s, x, xh, y, n_rows, d, n_classes);

    sof_data data;
    memset(&data, 0, sizeof(data));
    if (user) {
        data = *user;
        data.n_rows = n_rows;   // the frontiers use rows 0 .. n_rows-1 only
    } else {
        data.x = dtype == SOF_F16 ? (const void*)xh : (const void*)x;
        data.y = y;
        data.ld = n_rows;
        data.n_rows = n_rows;
        data.n_features = d;
        data.n_classes = n_classes;
        data.dtype = dtype;
    }

    // workspace for the largest frontier
    size_t ws_bytes = 0;
    for (int i = 0; i < n_sizes; ++i) {
        int N = n_rows / kSizes[i];
        if (N < 1) continue;
        if (kSizes[i] > kSmallMaxMin && kSizes[i] <= kMidSplit && N < n_tile) N = n_tile;
        sof_frontier fr{no, idx, (int64_t)N * kSizes[i], N, kSizes[i]};
        sof_proj pj{po, zo, zf, zw, (int64_t)N * kk * nnz, N * kk, kk};
        sof_params q{nullptr, bins, 0};
        size_t b = 0;
        int rc = sof_workspace_size(ctx, &data, &fr, &pj, &q, &b);
        if (rc) return rc;
        ws_bytes = b > ws_bytes ? b : ws_bytes;
    }
    void* ws;
    if ((e = B.get((char**)&ws, ws_bytes))) return hip_fail(e, "sof_autotune: hipMalloc");
    hipEvent_t ev0, ev1;
    if ((e = hipEventCreate(&ev0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&ev1)) != hipSuccess) {
        (void)hipEventDestroy(ev0);
        return hip_fail(e, "hipEventCreate");
    }
    float* half_us = out->half_us;
    int rc = SOF_OK;
    const int half_bins = bins / 2 >= SOF_MIN_BINS ? bins / 2 : SOF_MIN_BINS;
    bool warm[4] = {false, false, false, false};
    int hist_wins = 0;   // consecutive sizes at which histograms were not slower
    int np = 0;
    for (int i = 0; i < n_sizes && rc == SOF_OK; ++i) {
        const int sz = kSizes[i], N = n_rows / sz;
        if (N < 1) break;
        hipLaunchKernelGGL(k_tune_frontier, dim3(512), dim3(256), 0, s, no, idx, po, zo, zf, zw, N, sz, kk, nnz, d,
                           n_rows);
        sof_frontier fr{no, idx, (int64_t)N * sz, N, sz};
        sof_proj pj{po, zo, zf, zw, (int64_t)N * kk * nnz, N * kk, kk};
        float best[4] = {1e30f, 1e30f, 1e30f, 1e30f};
        const bool need_sort = hist_wins < 2, need_half = sz <= 1024;
        // the other wave tile of this size: a block per 4 projections instead
        // of a wave per projection (257..512), or 32 samples per thread
        // instead of 16 (2049..4096)
        const bool tile_small = sz > kSmallMaxMin && sz <= kSmallMax;
        const bool tile_mid = sz > kMidSplitMin && sz <= kMidSplit;
        // best of two timed calls (after a warm-up call when warm is false)
        auto time_calls = [&](const sof_frontier& f, const sof_proj& pp, const sof_params& q, bool warm) {
            float b = 1e30f;
            for (int rep = warm ? 1 : 0; rep < 3 && rc == SOF_OK; ++rep) {
                (void)hipEventRecord(ev0, s);
                rc = sof_find_splits(ctx, &data, &f, &pp, &q, sp, nullptr, ws, ws_bytes, stream);
                (void)hipEventRecord(ev1, s);
                if (rc) break;
                if ((e = hipEventSynchronize(ev1)) != hipSuccess) {
                    rc = hip_fail(e, "hipEventSynchronize");
                    break;
                }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, ev0, ev1);
                if (rep > 0 && ms < b) b = ms;
            }
            return b;
        };
        for (int path = 0; path < 3 && rc == SOF_OK; ++path) {
            // 0: sort path, 1: histogram path, 2: histogram path with half the bins
            if ((path == 0 && !need_sort) || (path == 2 && !need_half)) continue;
            sof_params q{nullptr, path == 2 ? half_bins : bins, path == 0 ? 0x7fffffff : 0};
            best[path] = time_calls(fr, pj, q, warm[path]);
            warm[path] = true;
        }
        const float per = 1e3f / (float)((int64_t)N * kk);   // ms per call -> us per node-projection
        out->sizes[i] = sz;
        out->hist_us[i] = best[1] * per;
        // not sorted: histograms had won at two smaller sizes (recorded as 0)
        out->sort_us[i] = need_sort ? best[0] * per : 0.f;
        // above 1024 samples half bins are not measured: recorded as full bins
        half_us[i] = need_half ? best[2] * per : out->hist_us[i];
        if ((tile_small || tile_mid) && rc == SOF_OK) {
            // both wave tiles on a frontier of at least n_tile nodes
            const int Nt = N > n_tile ? N : n_tile;
            hipLaunchKernelGGL(k_tune_frontier, dim3(512), dim3(256), 0, s, no, idx, po, zo, zf, zw, Nt, sz, kk,
                               nnz, d, n_rows);
            sof_frontier ft{no, idx, (int64_t)Nt * sz, Nt, sz};
            sof_proj pt{po, zo, zf, zw, (int64_t)Nt * kk * nnz, Nt * kk, kk};
            sof_params q{nullptr, bins, 0};
            const float base = time_calls(ft, pt, q, warm[3]);
            q.small_max = tile_small ? kSmallMaxMin : 0;
            q.mid_split = tile_mid ? kMidSplitMin : 0;
            best[3] = time_calls(ft, pt, q, warm[3]);
            warm[3] = true;
            const float pt_us = 1e3f / (float)((int64_t)Nt * kk);
            out->tile_base_us[i] = base * pt_us;
            out->tile_us[i] = best[3] * pt_us;
        }
        if (need_sort) hist_wins = out->hist_us[i] <= out->sort_us[i] ? hist_wins + 1 : 0;
        np = i + 1;
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (rc) return rc;
    out->n_points = np;
    // T: smallest size from which the histogram path is never slower (sizes
    // not sorted count as histogram wins)
    int T = SOF_SORT_LIMIT + 1;
    for (int i = np - 1; i >= 0; --i) {
        if (out->sort_us[i] == 0.f || out->hist_us[i] <= out->sort_us[i]) T = kSizes[i];
        else break;
    }
    out->sort_threshold = T;
    // bins switch: smallest size from which full bins cost at most 10% more than
    // half bins at every larger measured size (half bins below it); if the
    // largest size already fails, every measured size takes half bins
    int sw = np > 0 ? kSizes[np - 1] + 1 : 0;
    for (int i = np - 1; i >= 0; --i) {
        if (out->hist_us[i] <= 1.1f * half_us[i]) sw = kSizes[i];
        else break;
    }
    if (np > 0 && sw == kSizes[0]) sw = 0;
    out->bins_small = half_bins;
    out->bins_switch = sw;
    // wave tile edges: from the largest measured size of each range down, a
    // size whose other tile is more than 5% faster moves the edge below it
    int small_max = kSmallMax, mid_split = kMidSplit;
    for (int i = np - 1; i >= 0; --i) {
        const int sz = kSizes[i];
        if (sz > kSmallMaxMin && sz <= kSmallMax && sz == small_max && out->tile_us[i] > 0.f &&
            out->tile_us[i] * 1.05f < out->tile_base_us[i])
            small_max = i > 0 && kSizes[i - 1] >= kSmallMaxMin ? kSizes[i - 1] : kSmallMaxMin;
        if (sz > kMidSplitMin && sz <= kMidSplit && sz == mid_split && out->tile_us[i] > 0.f &&
            out->tile_us[i] * 1.05f < out->tile_base_us[i])
            mid_split = i > 0 && kSizes[i - 1] >= kMidSplitMin ? kSizes[i - 1] : kMidSplitMin;
    }
    out->small_max = small_max;
    out->mid_split = mid_split;
    out->elapsed_ms =
        std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - wall0).count();
    return SOF_OK;
}

extern "C" int sof_autotune(sof_ctx* ctx, int32_t dtype, int32_t n_classes, int32_t k, int32_t nnz,
                            int32_t bins, sof_tune* out, void* stream) {
    return autotune_impl(ctx, nullptr, dtype, n_classes, k, nnz, bins, out, stream);
}

extern "C" int sof_autotune_on(sof_ctx* ctx, const sof_data* data, int32_t k, int32_t nnz, int32_t bins,
                               sof_tune* out, void* stream) {
    int rc;
    if ((rc = check_data(data))) return rc;
    return autotune_impl(ctx, data, data->dtype, data->n_classes, k, nnz, bins, out, stream);
}
