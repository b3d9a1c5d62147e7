// k_grow.hip -- level-wise growth of several trees to purity (paper section
// 2: trees trained to purity; section 4.1: per-node switch between histograms
// and sorting; section 6: batching many nodes, here every node of every tree
// at one depth, into single launches).
//
// One level, all sizes read from device counters (so the sequence can be
// captured once in a HIP graph and replayed):
//   find splits      projections drawn on the fly (counter hash + Floyd)
//   partition        stable left/right blocks per node
//   k_gzero, k_gcount  class counts of every child segment -> labels
//   k_glevel         per node: children made, next-frontier nodes and samples
//   scans            exclusive scans of those counts (deterministic ids)
//   k_gwrite         node records, next frontier (offsets, tree, position)
//   k_gcopy          copy surviving children's samples into the next frontier
//   k_gfinish        advance counters, next tree starts
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "sof.h"
#include "sof_device.h"
#include "sof_host.h"
#include "sof_internal.h"
#include "sof_sampler.h"

namespace sof {

enum { G_NFRONT = 0, G_LEVEL = 1, G_NNODES = 2, G_NEXTN = 3, G_NSAMP = 4, G_COUNT = 8 };

struct GrowArgs {
    const int32_t* y;
    int32_t n_rows, n_classes, n_trees, k, z, n_features, max_depth, bins;
    int32_t sampler, weights;     // SOF_SAMPLER_*, SOF_WEIGHTS_*
    int32_t first_tree;           // f_tree / n_tree hold tree ids first_tree .. first_tree + n_trees - 1
    uint64_t seed;
    int32_t* cnt;                 // G_* counters
    const int32_t* f_off;         // current frontier
    const int32_t* f_idx;
    const int32_t* f_node;
    const int32_t* f_tree;
    const int32_t* f_pos;
    const int32_t* f_tstart;      // n_trees + 1, indexed by tree id - first_tree
    int32_t* n_off;               // next frontier
    int32_t* n_idx;
    int32_t* n_node;
    int32_t* n_tree;
    int32_t* n_pos;
    int32_t* n_tstart;
    int32_t* n_src;               // next node -> start of its block in part_idx
    const void* splits;           // SplitRec
    const int32_t* part_idx;
    const int32_t* child_off;     // 2N + 1
    int32_t* child_cnt;           // 2 * cap * classes
    int64_t* scan_a;              // cap + 1: children << 32 | next nodes
    int64_t* scan_b;              // cap + 1: next samples
    int64_t* blk;                 // scan block sums
    sof_tree_node* nodes;
    int64_t cap_front, cap_nodes, n_samples;
};

__device__ __forceinline__ int gN(const GrowArgs& g) {
    int n = g.cnt[G_NFRONT];
    return n < 0 ? 0 : (n > g.cap_front ? (int)g.cap_front : n);
}

// The winning projection of a node into its record: features ascending,
// FP32 weights, zeros past nnz.
__device__ void g_sample(const GrowArgs& g, int tree, int level, int pos, int p, sof_tree_node& nd) {
    const SampSpec sp{g.seed, g.n_features, g.z, g.sampler, g.weights};
    int32_t f[SOF_MAX_NNZ];
    uint32_t w[SOF_MAX_NNZ];
    const int z = samp_thread(sp, tree, level, pos, p, f, w);
    nd.nnz = z;
    for (int q = 0; q < SOF_MAX_NNZ; ++q) {
        nd.feature[q] = q < z ? f[q] : 0;
        nd.weight[q] = q < z ? __uint_as_float(w[q]) : 0.f;
    }
}

// Work over the concatenation of M contiguous segments [off[j], off[j+1])
// (monotone offsets from 0): each wave takes chunks of kSegChunk positions and
// walks the segments a chunk overlaps, so one huge segment and many tiny ones
// both spread over the whole grid.
constexpr int kSegChunk = 2048;

// the segment that holds position pos, for off[0] <= pos < off[M]: the last j
// with off[j] <= pos (empty segments before it are skipped)
__device__ __forceinline__ int seg_find(const int32_t* off, int M, int64_t pos) {
    int lo = 0, hi = M - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= pos) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// zero the class counts that k_gcount accumulates into (a kernel rather than
// a memset node, so that graph replays stay exact)
__global__ __launch_bounds__(256) void k_gzero(GrowArgs g, int use_children) {
    const int N = gN(g);
    const int64_t n = (int64_t)(use_children ? 2 * N : N) * g.n_classes;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) g.child_cnt[i] = 0;
}

// class counts of M consecutive segments of idx (children after the
// partition, or the roots): per 64 positions one ballot per class, then one
// atomic add per (segment, class) per chunk
__global__ __launch_bounds__(256) void k_gcount(GrowArgs g, int use_children) {
    const int N = gN(g);
    const int M = use_children ? 2 * N : N;
    if (M <= 0) return;
    const int32_t* off = use_children ? g.child_off : g.f_off;
    const int32_t* idx = use_children ? g.part_idx : g.f_idx;
    const int lane = threadIdx.x & 63;
    const int C = g.n_classes;
    int64_t total = __builtin_amdgcn_readfirstlane(off[M]);
    if (total > g.n_samples) total = g.n_samples;
    const int64_t waves = (int64_t)gridDim.x * 4;
    // every loop bound below is a scalar, so the lane-subset atomic at the end
    // of an iteration closes before the next iteration's ballots
    const int wave = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * 256 + threadIdx.x) >> 6));
    for (int64_t ch = wave; ch * kSegChunk < total; ch += waves) {
        const int64_t cs = ch * kSegChunk;
        const int64_t ce = cs + kSegChunk < total ? cs + kSegChunk : total;
        for (int j = __builtin_amdgcn_readfirstlane(seg_find(off, M, cs)); j < M; ++j) {
            const int64_t o0 = __builtin_amdgcn_readfirstlane(off[j]);
            const int64_t o1 = __builtin_amdgcn_readfirstlane(off[j + 1]);
            const int64_t a = o0 > cs ? o0 : cs;
            const int64_t b = o1 < ce ? o1 : ce;
            uint32_t cnt[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) cnt[c] = 0;
            for (int64_t i0 = a; i0 < b; i0 += 64) {
                const int64_t i = i0 + lane;
                uint32_t yv = 16;
                if (i < b) {
                    const uint32_t r = (uint32_t)idx[i];
                    yv = (uint32_t)g.y[r < (uint32_t)g.n_rows ? r : 0];
                    yv = yv < (uint32_t)C ? yv : 0;
                }
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    if (c < C) cnt[c] += (uint32_t)__popcll(__ballot(yv == (uint32_t)c));
            }
            uint32_t mine = 0;
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (lane == c) mine = cnt[c];
            if (lane < C && mine) atomicAdd(&g.child_cnt[(int64_t)j * C + lane], (int32_t)mine);
            if (o1 >= ce) break;
        }
    }
}

__device__ __forceinline__ int majority(const int32_t* cnt, int C) {
    int best = 0;
    for (int c = 1; c < C; ++c)
        if (cnt[c] > cnt[best]) best = c;
    return best;
}

// per frontier node: number of children made and of next-frontier nodes/samples
__global__ __launch_bounds__(256) void k_glevel(GrowArgs g) {
    const int N = gN(g);
    const int level = g.cnt[G_LEVEL];
    for (int v = blockIdx.x * 256 + threadIdx.x; v <= N; v += gridDim.x * 256) {
        if (v == N) { g.scan_a[v] = 0; g.scan_b[v] = 0; continue; }
        const SplitRec s = ((const SplitRec*)g.splits)[v];
        int64_t children = 0, nn = 0, ns = 0;
        if (s.proj >= 0) {
            children = 2;
            const int32_t nc[2] = {s.n_left, s.n_right};
            for (int c = 0; c < 2; ++c) {
                bool pure = (s.flags >> c) & 1;
                bool leaf = nc[c] < 2 || pure || level + 1 >= g.max_depth;
                if (!leaf) { nn += 1; ns += nc[c]; }
            }
        }
        g.scan_a[v] = (children << 32) | nn;
        g.scan_b[v] = ns;
    }
}

// exclusive scan over N+1 int64 entries, N read from the device (three kernels)
constexpr int kScanBlock = 1024;

__device__ __forceinline__ int64_t wave_scan64(int64_t x) {
    const int lane = threadIdx.x & 63;
    for (int off = 1; off < 64; off <<= 1) {
        int64_t t = __shfl_up(x, off);
        if (lane >= off) x += t;
    }
    return x;
}

__global__ __launch_bounds__(kScanBlock) void k_scan1(const int32_t* cnt, int64_t* a, int64_t* blk) {
    extern __shared__ __align__(16) char smem[];
    int64_t* part = (int64_t*)smem;
    const int n = cnt[G_NFRONT] + 1;
    const int nb = (n + kScanBlock - 1) / kScanBlock;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        const int i = b * kScanBlock + threadIdx.x;
        int64_t x = i < n ? a[i] : 0;
        int64_t incl = wave_scan64(x);
        if ((threadIdx.x & 63) == 63) part[threadIdx.x >> 6] = incl;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t t = 0;
            for (int w = 0; w < kScanBlock / 64; ++w) t += part[w];
            blk[b] = t;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan2(const int32_t* cnt, int64_t* blk) {
    extern __shared__ __align__(16) char smem[];
    int64_t* part = (int64_t*)smem;     // 16 wave totals + carry
    const int n = cnt[G_NFRONT] + 1;
    const int nb = (n + kScanBlock - 1) / kScanBlock;
    int64_t carry = 0;
    for (int base = 0; base < nb; base += kScanBlock) {
        const int i = base + threadIdx.x;
        int64_t x = i < nb ? blk[i] : 0;
        int64_t incl = wave_scan64(x);
        if ((threadIdx.x & 63) == 63) part[threadIdx.x >> 6] = incl;
        __syncthreads();
        int64_t before = carry, tot = carry;
        for (int w = 0; w < kScanBlock / 64; ++w) {
            if (w < (int)(threadIdx.x >> 6)) before += part[w];
            tot += part[w];
        }
        if (i < nb) blk[i] = before + incl - x;
        carry = tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan3(const int32_t* cnt, int64_t* a, const int64_t* blk) {
    extern __shared__ __align__(16) char smem[];
    int64_t* part = (int64_t*)smem;
    const int n = cnt[G_NFRONT] + 1;
    const int nb = (n + kScanBlock - 1) / kScanBlock;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        const int i = b * kScanBlock + threadIdx.x;
        int64_t x = i < n ? a[i] : 0;
        int64_t incl = wave_scan64(x);
        if ((threadIdx.x & 63) == 63) part[threadIdx.x >> 6] = incl;
        __syncthreads();
        int64_t before = blk[b];
        for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) before += part[w];
        if (i < n) a[i] = before + incl - x;
        __syncthreads();
    }
}

// node records of split nodes and of their children; next-frontier entries
__global__ __launch_bounds__(256) void k_gwrite(GrowArgs g) {
    const int N = gN(g);
    const int level = g.cnt[G_LEVEL];
    const int64_t base_nodes = g.cnt[G_NNODES];
    const int C = g.n_classes;
    for (int v = blockIdx.x * 256 + threadIdx.x; v < N; v += gridDim.x * 256) {
        const SplitRec s = ((const SplitRec*)g.splits)[v];
        const int me = g.f_node[v];
        if (me < 0 || me >= g.cap_nodes) continue;
        sof_tree_node& nd = g.nodes[me];
        if (s.proj < 0) {
            nd.is_leaf = 1;
            nd.kind = -1;
            continue;
        }
        const int tree = g.f_tree[v];
        const int64_t a = g.scan_a[v];
        const int64_t lid = base_nodes + (a >> 32);
        if (lid + 2 > g.cap_nodes) continue;
        nd.is_leaf = 0;
        nd.kind = s.kind;
        nd.bin = s.bin;
        nd.threshold = s.threshold;
        nd.lo = s.lo;
        nd.scale = s.scale;
        nd.gain = (double)s.gain;
        nd.n_bins = g.bins;
        nd.left = (int32_t)lid;
        nd.right = (int32_t)(lid + 1);
        g_sample(g, tree, level, g.f_pos[v], s.proj, nd);
        int64_t next = a & 0xffffffffll;
        int64_t nbase = g.scan_b[v];
        const int32_t nc[2] = {s.n_left, s.n_right};
        for (int c = 0; c < 2; ++c) {
            sof_tree_node& ch = g.nodes[lid + c];
            const int32_t* cc = g.child_cnt + (int64_t)(2 * v + c) * C;
            bool pure = (s.flags >> c) & 1;
            bool leaf = nc[c] < 2 || pure || level + 1 >= g.max_depth;
            ch.tree = tree;
            ch.depth = level + 1;
            ch.parent = me;
            ch.left = -1;
            ch.right = -1;
            ch.n_samples = nc[c];
            ch.label = majority(cc, C);
            ch.is_leaf = leaf ? 1 : 0;
            ch.kind = -1;
            ch.bin = -1;
            ch.threshold = 0.f;
            ch.lo = 0.f;
            ch.scale = 0.f;
            ch.n_bins = 0;
            ch.nnz = 0;
            ch.pad = 0;
            for (int q = 0; q < 16; ++q) { ch.feature[q] = 0; ch.weight[q] = 0.f; }
            ch.gain = 0.0;
            if (!leaf && next < g.cap_front) {
                g.n_off[next] = (int32_t)nbase;
                g.n_node[next] = (int32_t)(lid + c);
                g.n_tree[next] = tree;
                g.n_src[next] = g.child_off[2 * v + c];
                next += 1;
                nbase += nc[c];
            }
        }
    }
}

// next frontier: offsets end, positions within trees, tree starts, sample copy
__global__ __launch_bounds__(256) void k_gnext(GrowArgs g) {
    const int N = gN(g);
    const int64_t nn = g.scan_a[N] & 0xffffffffll;
    if (blockIdx.x == 0)
        for (int t = threadIdx.x; t <= g.n_trees; t += blockDim.x) {
            int ts = g.f_tstart[t];
            ts = ts < 0 ? 0 : (ts > N ? N : ts);
            g.n_tstart[t] = (int32_t)(g.scan_a[ts] & 0xffffffffll);
        }
    if (blockIdx.x == 0 && threadIdx.x == 0) g.n_off[nn] = (int32_t)g.scan_b[N];
    // positions: the index of each next node within its tree's run; runs are
    // contiguous and ordered by tree, so pos = j - (first j of that tree)
    for (int64_t j = blockIdx.x * 256 + threadIdx.x; j < nn; j += gridDim.x * 256) {
        // local index of the node's tree (tree ids start at first_tree)
        int t = g.n_tree[j] - g.first_tree;
        t = t < 0 ? 0 : (t >= g.n_trees ? g.n_trees - 1 : t);
        // first next index of tree t = scan_a low part at the tree's first current node
        int ts = g.f_tstart[t];
        ts = ts < 0 ? 0 : (ts > N ? N : ts);
        g.n_pos[j] = (int32_t)(j - (g.scan_a[ts] & 0xffffffffll));
    }
}

// copy the surviving children's sample blocks into the next frontier, chunked
// over the destination positions like k_gcount
__global__ __launch_bounds__(256) void k_gcopy(GrowArgs g) {
    const int N = gN(g);
    int64_t nn = g.scan_a[N] & 0xffffffffll;
    if (nn <= 0 || nn > g.cap_front) return;
    const int M = (int)nn;
    const int lane = threadIdx.x & 63;
    int64_t total = g.n_off[M];
    if (total > g.n_samples) total = g.n_samples;
    const int64_t waves = (int64_t)gridDim.x * 4;
    for (int64_t ch = (blockIdx.x * 256 + threadIdx.x) >> 6; ch * kSegChunk < total; ch += waves) {
        const int64_t cs = ch * kSegChunk;
        const int64_t ce = cs + kSegChunk < total ? cs + kSegChunk : total;
        for (int j = seg_find(g.n_off, M, cs); j < M; ++j) {
            const int64_t d0 = g.n_off[j], d1 = g.n_off[j + 1];
            const int64_t s0 = g.n_src[j];
            if (!(d0 < 0 || d1 > g.n_samples || d1 < d0 || s0 < 0 || s0 + (d1 - d0) > g.n_samples)) {
                const int64_t a = d0 > cs ? d0 : cs;
                const int64_t b = d1 < ce ? d1 : ce;
                for (int64_t i = a + lane; i < b; i += 64) g.n_idx[i] = g.part_idx[s0 + (i - d0)];
            }
            if (d1 >= ce) break;
        }
    }
}

__global__ void k_gfinish(GrowArgs g) {
    if (threadIdx.x != 0) return;
    const int N = gN(g);
    const int64_t a = g.scan_a[N];
    g.cnt[G_NNODES] += (int32_t)(a >> 32);
    g.cnt[G_NEXTN] = (int32_t)(a & 0xffffffffll);
    g.cnt[G_NFRONT] = (int32_t)(a & 0xffffffffll);
    g.cnt[G_NSAMP] = (int32_t)g.scan_b[N];
    g.cnt[G_LEVEL] += 1;
}

// ---------------------------------------------------------------------------
// host side

struct GrowBuffers {
    int32_t* off[2];
    int32_t* idx[2];
    int32_t* node[2];
    int32_t* tree[2];
    int32_t* pos[2];
    int32_t* tstart[2];
    int32_t* src;
    int32_t* cnt;
    void* splits;
    int32_t* part_idx;
    int32_t* child_off;
    int32_t* child_cnt;
    int64_t* scan_a;
    int64_t* scan_b;
    int64_t* blk;
    sof_tree_node* nodes;
    void* ws_find;
    void* ws_part;
};

}  // namespace sof

using namespace sof;

struct sof_forest {
    sof_ctx* ctx = nullptr;
    sof_data data;
    sof_forest_desc desc;
    std::vector<int64_t> root_off;
    int64_t n_samples = 0, cap_front = 0, cap_nodes = 0;
    GrowBuffers b;
    std::vector<void*> allocs;
    FindLayout flay;
    int cur = 0;
    int level = 0;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    LaunchCfg cfg;
};

static int falloc(sof_forest* f, void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes < 256 ? 256 : bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc (forest)");
    f->allocs.push_back(*p);
    return SOF_OK;
}

static GrowArgs grow_args(sof_forest* f) {
    GrowArgs g;
    memset(&g, 0, sizeof(g));
    const int c = f->cur, n = 1 - c;
    g.y = f->data.y;
    g.n_rows = f->data.n_rows;
    g.n_classes = f->data.n_classes;
    g.n_trees = f->desc.n_trees;
    g.k = f->desc.k;
    g.z = f->desc.z;
    g.n_features = f->data.n_features;
    g.max_depth = f->desc.max_depth;
    g.bins = f->desc.bins;
    g.seed = f->desc.seed;
    g.sampler = f->desc.sampler;
    g.weights = f->desc.weights;
    g.first_tree = f->desc.first_tree;
    g.cnt = f->b.cnt;
    g.f_off = f->b.off[c];
    g.f_idx = f->b.idx[c];
    g.f_node = f->b.node[c];
    g.f_tree = f->b.tree[c];
    g.f_pos = f->b.pos[c];
    g.f_tstart = f->b.tstart[c];
    g.n_off = f->b.off[n];
    g.n_idx = f->b.idx[n];
    g.n_node = f->b.node[n];
    g.n_tree = f->b.tree[n];
    g.n_pos = f->b.pos[n];
    g.n_tstart = f->b.tstart[n];
    g.n_src = f->b.src;
    g.splits = f->b.splits;
    g.part_idx = f->b.part_idx;
    g.child_off = f->b.child_off;
    g.child_cnt = f->b.child_cnt;
    g.scan_a = f->b.scan_a;
    g.scan_b = f->b.scan_b;
    g.blk = f->b.blk;
    g.nodes = f->b.nodes;
    g.cap_front = f->cap_front;
    g.cap_nodes = f->cap_nodes;
    g.n_samples = f->n_samples;
    return g;
}

// one level on stream s (no allocation, no synchronisation)
static hipError_t level_launch(sof_forest* f, hipStream_t s) {
    const int c = f->cur;
    GrowArgs g = grow_args(f);
    FindArgs a;
    memset(&a, 0, sizeof(a));
    a.x = f->data.x;
    a.ld = f->data.ld;
    a.y = f->data.y;
    a.n_rows = f->data.n_rows;
    a.n_features = f->data.n_features;
    a.n_classes = f->data.n_classes;
    a.dtype = f->data.dtype;
    a.node_offsets = f->b.off[c];
    a.sample_idx = f->b.idx[c];
    a.n_samples = f->n_samples;
    a.n_nodes = (int32_t)f->cap_front;
    a.n_nodes_dev = f->b.cnt + G_NFRONT;
    a.node_bins = nullptr;
    a.bins = f->desc.bins;
    a.sort_threshold = clamp_threshold(f->desc.sort_threshold);
    a.small_max = kSmallMax;
    a.mid_split = kMidSplit;
    a.bin_mode = f->desc.bin_mode;
    a.criterion = f->desc.criterion;
    a.bin_seed = f->desc.bin_seed;
    a.out = f->b.splits;
    a.hist_out = nullptr;
    find_bind(f->flay, f->b.ws_find, &a.ws);
    ProjHash ph{f->b.tree[c], f->b.pos[c], f->b.cnt + G_LEVEL, f->desc.seed, f->desc.k, f->desc.z,
                f->desc.sampler, f->desc.weights};
    hipError_t e = launch_find_hash(a, ph, f->cfg, find_streams(f->ctx, s));
    if (e != hipSuccess) return e;
    PartArgs pa;
    memset(&pa, 0, sizeof(pa));
    pa.x = f->data.x;
    pa.ld = f->data.ld;
    pa.n_rows = f->data.n_rows;
    pa.n_features = f->data.n_features;
    pa.dtype = f->data.dtype;
    pa.node_offsets = f->b.off[c];
    pa.sample_idx = f->b.idx[c];
    pa.n_samples = f->n_samples;
    pa.n_nodes = (int32_t)f->cap_front;
    pa.n_nodes_dev = f->b.cnt + G_NFRONT;
    pa.node_bins = nullptr;
    pa.bins = f->desc.bins;
    pa.splits = f->b.splits;
    pa.out_idx = f->b.part_idx;
    pa.child_offsets = f->b.child_off;
    part_bind(f->cap_front, f->n_samples, f->b.ws_part, &pa);
    e = launch_partition_hash(pa, ph, f->ctx->n_cu, find_streams(f->ctx, s));
    if (e != hipSuccess) return e;
    const int grid = f->ctx->n_cu * 4;
    const int nb_scan = (int)((f->cap_front + 1 + kScanBlock - 1) / kScanBlock);
    const int g_scan = nb_scan < grid ? nb_scan : grid;
    hipLaunchKernelGGL(k_gzero, dim3(grid), dim3(256), 0, s, g, 1);
    hipLaunchKernelGGL(k_gcount, dim3(grid), dim3(256), 0, s, g, 1);
    hipLaunchKernelGGL(k_glevel, dim3(grid), dim3(256), 0, s, g);
    for (int64_t* arr : {g.scan_a, g.scan_b}) {
        hipLaunchKernelGGL(k_scan1, dim3(g_scan), dim3(kScanBlock), 16 * sizeof(int64_t), s, (const int32_t*)g.cnt, arr, g.blk);
        hipLaunchKernelGGL(k_scan2, dim3(1), dim3(kScanBlock), 16 * sizeof(int64_t), s, (const int32_t*)g.cnt, g.blk);
        hipLaunchKernelGGL(k_scan3, dim3(g_scan), dim3(kScanBlock), 16 * sizeof(int64_t), s, (const int32_t*)g.cnt, arr, (const int64_t*)g.blk);
    }
    hipLaunchKernelGGL(k_gwrite, dim3(grid), dim3(256), 0, s, g);
    hipLaunchKernelGGL(k_gnext, dim3(grid), dim3(256), 0, s, g);
    hipLaunchKernelGGL(k_gcopy, dim3(grid), dim3(256), 0, s, g);
    hipLaunchKernelGGL(k_gfinish, dim3(1), dim3(64), 0, s, g);
    return hipGetLastError();
}

static void forest_free(sof_forest* f) {
    for (int i = 0; i < 2; ++i)
        if (f->exec[i]) (void)hipGraphExecDestroy(f->exec[i]);
    if (f->cap_stream) (void)hipStreamDestroy(f->cap_stream);
    for (void* p : f->allocs) (void)hipFree(p);
    delete f;
}

extern "C" int sof_forest_create(sof_ctx* ctx, const sof_data* data, const sof_forest_desc* desc,
                                 sof_forest** out) {
    if (!ctx || !out) return fail(SOF_ERR_INVALID_ARG, "ctx or out is NULL");
    *out = nullptr;
    int rc;
    if ((rc = check_data(data))) return rc;
    if (!desc || !desc->root_offsets || !desc->root_idx) return fail(SOF_ERR_INVALID_ARG, "desc/roots NULL");
    if (desc->n_trees < 1 || desc->n_trees > 1024) return fail(SOF_ERR_INVALID_ARG, "n_trees %d", desc->n_trees);
    if (desc->first_tree < 0 || (int64_t)desc->first_tree + desc->n_trees > (1 << 20))
        return fail(SOF_ERR_INVALID_ARG, "tree ids out of range");
    if (desc->k < 1 || desc->k > 1024) return fail(SOF_ERR_INVALID_ARG, "k %d outside [1, 1024]", desc->k);
    if (desc->sampler != SOF_SAMPLER_FIXED && desc->sampler != SOF_SAMPLER_DENSITY)
        return fail(SOF_ERR_UNSUPPORTED, "sampler %d", desc->sampler);
    if (desc->weights != SOF_WEIGHTS_SIGN && desc->weights != SOF_WEIGHTS_UNIFORM)
        return fail(SOF_ERR_UNSUPPORTED, "weights %d", desc->weights);
    if (desc->sampler == SOF_SAMPLER_FIXED && (desc->z < 1 || desc->z > 15 || desc->z > data->n_features))
        return fail(SOF_ERR_INVALID_ARG, "z %d outside [1, min(15, n_features)]", desc->z);
    if (desc->sampler == SOF_SAMPLER_DENSITY && (desc->z < 1 || desc->z > SOF_MAX_NNZ))
        return fail(SOF_ERR_INVALID_ARG, "mean nonzeros z %d outside [1, %d]", desc->z, SOF_MAX_NNZ);
    if (desc->bins < 2 || desc->bins > SOF_MAX_BINS) return fail(SOF_ERR_UNSUPPORTED, "bins %d", desc->bins);
    if (desc->sort_threshold < 0) return fail(SOF_ERR_INVALID_ARG, "sort_threshold < 0");
    if (desc->max_depth < 0 || desc->max_depth > 64) return fail(SOF_ERR_INVALID_ARG, "max_depth %d", desc->max_depth);
    if (desc->criterion != SOF_CRIT_GINI && desc->criterion != SOF_CRIT_ENTROPY)
        return fail(SOF_ERR_UNSUPPORTED, "criterion %d", desc->criterion);
    if (desc->bin_mode != SOF_BINS_EQUAL && desc->bin_mode != SOF_BINS_RANDOM)
        return fail(SOF_ERR_UNSUPPORTED, "bin_mode %d", desc->bin_mode);
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    sof_forest* f = new sof_forest();
    f->ctx = ctx;
    f->data = *data;
    f->desc = *desc;
    f->root_off.assign(desc->root_offsets, desc->root_offsets + desc->n_trees + 1);
    if (f->root_off[0] != 0) { delete f; return fail(SOF_ERR_INVALID_ARG, "root_offsets[0] != 0"); }
    int64_t maxroot = 0;
    for (int t = 0; t < desc->n_trees; ++t) {
        int64_t n = f->root_off[t + 1] - f->root_off[t];
        if (n < 0) { delete f; return fail(SOF_ERR_INVALID_ARG, "root_offsets decrease"); }
        if (n > maxroot) maxroot = n;
    }
    f->n_samples = f->root_off[desc->n_trees];
    if (f->n_samples > 0x7fffffffLL) { delete f; return fail(SOF_ERR_OVERFLOW, "total root samples"); }
    if (maxroot > SOF_MAX_NODE_SAMPLES) { delete f; return fail(SOF_ERR_OVERFLOW, "root above 2^24 samples"); }
    f->cap_front = f->n_samples / 2 + desc->n_trees + 1;
    f->cap_nodes = 2 * f->n_samples + desc->n_trees + 2;
    const int mode = (desc->bin_mode == SOF_BINS_RANDOM ? 1 : 0) | (desc->criterion == SOF_CRIT_ENTROPY ? 2 : 0);
    if ((rc = launch_cfg(ctx, desc->bins, data->n_classes, mode, &f->cfg))) { delete f; return rc; }
    const int C = data->n_classes;
    const int64_t S = f->n_samples > 0 ? f->n_samples : 1, F = f->cap_front;
    f->flay = find_layout(F, S, F * desc->k, desc->k, desc->bins, C, flnk_entries(desc->criterion, maxroot));
    GrowBuffers& b = f->b;
    for (int i = 0; i < 2; ++i) {
        if ((rc = falloc(f, (void**)&b.off[i], (F + 1) * 4)) || (rc = falloc(f, (void**)&b.idx[i], S * 4)) ||
            (rc = falloc(f, (void**)&b.node[i], F * 4)) || (rc = falloc(f, (void**)&b.tree[i], F * 4)) ||
            (rc = falloc(f, (void**)&b.pos[i], F * 4)) || (rc = falloc(f, (void**)&b.tstart[i], (desc->n_trees + 1) * 4))) {
            forest_free(f);
            return rc;
        }
    }
    const int64_t nb = (F + 1 + kScanBlock - 1) / kScanBlock + 1;
    if ((rc = falloc(f, (void**)&b.src, F * 4)) || (rc = falloc(f, (void**)&b.cnt, G_COUNT * 4)) ||
        (rc = falloc(f, &b.splits, F * 40)) || (rc = falloc(f, (void**)&b.part_idx, S * 4)) ||
        (rc = falloc(f, (void**)&b.child_off, (2 * F + 1) * 4)) ||
        (rc = falloc(f, (void**)&b.child_cnt, (2 * F + 2) * C * 4)) ||
        (rc = falloc(f, (void**)&b.scan_a, (F + 1) * 8)) || (rc = falloc(f, (void**)&b.scan_b, (F + 1) * 8)) ||
        (rc = falloc(f, (void**)&b.blk, nb * 8)) ||
        (rc = falloc(f, (void**)&b.nodes, f->cap_nodes * sizeof(sof_tree_node))) ||
        (rc = falloc(f, &b.ws_find, f->flay.total)) ||
        (rc = falloc(f, &b.ws_part, part_workspace(F, S)))) {
        forest_free(f);
        return rc;
    }
    // roots: counts on the device, leaf decisions and records on the host
    const int T = desc->n_trees;
    std::vector<int32_t> off32(T + 1);
    for (int t = 0; t <= T; ++t) off32[t] = (int32_t)f->root_off[t];
    e = hipMemcpy(b.off[0], off32.data(), (T + 1) * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && f->n_samples > 0)
        e = hipMemcpy(b.idx[0], desc->root_idx, f->n_samples * 4, hipMemcpyDeviceToDevice);
    int32_t cnt0[G_COUNT] = {T, 0, 0, 0, 0, 0, 0, 0};
    if (e == hipSuccess) e = hipMemcpy(b.cnt, cnt0, sizeof(cnt0), hipMemcpyHostToDevice);
    if (e != hipSuccess) { forest_free(f); return hip_fail(e, "forest roots"); }
    GrowArgs g = grow_args(f);
    hipLaunchKernelGGL(k_gzero, dim3(ctx->n_cu), dim3(256), 0, nullptr, g, 0);
    hipLaunchKernelGGL(k_gcount, dim3(ctx->n_cu * 4), dim3(256), 0, nullptr, g, 0);
    std::vector<int32_t> cnt((size_t)T * C);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(cnt.data(), b.child_cnt, cnt.size() * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) { forest_free(f); return hip_fail(e, "root counts"); }
    std::vector<sof_tree_node> roots(T);
    std::vector<int32_t> foff(1, 0), fnode, ftree, fpos, tstart(T + 1, 0);
    std::vector<int64_t> copy_src;
    for (int t = 0; t < T; ++t) {
        sof_tree_node& r = roots[t];
        memset(&r, 0, sizeof(r));
        const int32_t* cc = cnt.data() + (size_t)t * C;
        int best = 0, nonzero = 0;
        for (int c = 0; c < C; ++c) {
            if (cc[c] > cc[best]) best = c;
            if (cc[c] > 0) ++nonzero;
        }
        const int64_t n = f->root_off[t + 1] - f->root_off[t];
        r.tree = desc->first_tree + t;
        r.depth = 0;
        r.parent = r.left = r.right = -1;
        r.n_samples = (int32_t)n;
        r.label = best;
        r.kind = -1;
        r.bin = -1;
        r.is_leaf = (n < 2 || nonzero <= 1 || desc->max_depth == 0) ? 1 : 0;
        tstart[t] = (int32_t)fnode.size();
        if (!r.is_leaf) {
            fnode.push_back(t);
            ftree.push_back(r.tree);
            fpos.push_back(0);
            copy_src.push_back(f->root_off[t]);
            foff.push_back(foff.back() + (int32_t)n);
        }
    }
    tstart[T] = (int32_t)fnode.size();
    const int N0 = (int)fnode.size();
    e = hipMemcpy(b.nodes, roots.data(), T * sizeof(sof_tree_node), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b.off[0], foff.data(), (N0 + 1) * 4, hipMemcpyHostToDevice);
    for (int v = 0; v < N0 && e == hipSuccess; ++v)
        e = hipMemcpy(b.idx[0] + foff[v], desc->root_idx + copy_src[v], (size_t)(foff[v + 1] - foff[v]) * 4,
                      hipMemcpyDeviceToDevice);
    if (e == hipSuccess && N0 > 0) e = hipMemcpy(b.node[0], fnode.data(), N0 * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && N0 > 0) e = hipMemcpy(b.tree[0], ftree.data(), N0 * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && N0 > 0) e = hipMemcpy(b.pos[0], fpos.data(), N0 * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b.tstart[0], tstart.data(), (T + 1) * 4, hipMemcpyHostToDevice);
    int32_t cnt1[G_COUNT] = {N0, 0, T, 0, foff.back(), 0, 0, 0};
    if (e == hipSuccess) e = hipMemcpy(b.cnt, cnt1, sizeof(cnt1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) { forest_free(f); return hip_fail(e, "forest setup"); }
    *out = f;
    return SOF_OK;
}

extern "C" int sof_forest_destroy(sof_forest* f) {
    if (f) forest_free(f);
    return SOF_OK;
}

extern "C" int sof_grow_level(sof_forest* f, int use_graph, void* stream) {
    if (!f) return fail(SOF_ERR_INVALID_ARG, "forest is NULL");
    hipError_t e = hipSetDevice(f->ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    if (!use_graph) {
        {
            std::lock_guard<std::mutex> g(f->ctx->launch_mu);
            e = level_launch(f, s);
        }
        if (e != hipSuccess) return hip_fail(e, "grow_level launch");
    } else {
        const int c = f->cur;
        if (!f->exec[c]) {
            if (!f->cap_stream) {
                e = hipStreamCreateWithFlags(&f->cap_stream, hipStreamNonBlocking);
                if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
            }
            hipGraph_t graph = nullptr;
            e = hipStreamBeginCapture(f->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
            hipError_t le;
            {
                std::lock_guard<std::mutex> g(f->ctx->launch_mu);
                le = level_launch(f, f->cap_stream);
                e = hipStreamEndCapture(f->cap_stream, &graph);
            }
            if (le != hipSuccess) return hip_fail(le, "grow_level capture");
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&f->exec[c], graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        }
        e = hipGraphLaunch(f->exec[c], s);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    }
    f->cur = 1 - f->cur;
    f->level += 1;
    return SOF_OK;
}

extern "C" int sof_forest_frontier_size(sof_forest* f, int64_t* n, void* stream) {
    if (!f || !n) return fail(SOF_ERR_INVALID_ARG, "NULL argument");
    int32_t v = 0;
    hipError_t e = hipMemcpyAsync(&v, f->b.cnt + G_NFRONT, 4, hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "frontier size");
    *n = v;
    return SOF_OK;
}

extern "C" int sof_forest_frontier_stats(sof_forest* f, int64_t* n_nodes, int64_t* n_samples, int32_t* depth,
                                         void* stream) {
    if (!f || !n_nodes || !n_samples || !depth) return fail(SOF_ERR_INVALID_ARG, "NULL argument");
    int32_t cnt[G_COUNT];
    hipError_t e = hipMemcpyAsync(cnt, f->b.cnt, sizeof(cnt), hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "frontier stats");
    *n_nodes = cnt[G_NFRONT];
    *n_samples = cnt[G_NFRONT] > 0 ? cnt[G_NSAMP] : 0;
    *depth = cnt[G_LEVEL];
    return SOF_OK;
}

extern "C" int sof_forest_export(sof_forest* f, sof_tree_node* host, int64_t cap, int64_t* n, void* stream) {
    if (!f || !n) return fail(SOF_ERR_INVALID_ARG, "NULL argument");
    int32_t cnt[G_COUNT];
    hipError_t e = hipMemcpyAsync(cnt, f->b.cnt, sizeof(cnt), hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "export counters");
    *n = cnt[G_NNODES];
    if (!host || cap < *n) return fail(SOF_ERR_INVALID_ARG, "export: capacity %lld < %lld nodes", (long long)cap, (long long)*n);
    e = hipMemcpyAsync(host, f->b.nodes, (size_t)*n * sizeof(sof_tree_node), hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "export nodes");
    return SOF_OK;
}
