// sof_internal.h -- host/device plumbing shared by the library's translation
// units: argument blocks, work-queue layout and launch entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "sof.h"

namespace sof {

// Size classes of the batched frontier launch.  A node takes the sort path
// when n < T (T clamped to SOF_SORT_LIMIT + 1), else the histogram path.
constexpr int kSortWaveMax = 64;     // sort nodes up to here: sorted in registers by one wave
constexpr int kSmallMax = 512;       // histogram nodes up to here: one block per node (8 samples per lane)
constexpr int kMidSplit = 4096;      // mid nodes up to here: at most 16 samples per thread
constexpr int kMidMax = 8192;        // histogram nodes up to here: one block per (node, projection group)
// ranges of the run-time wave tile edges (sof_params.small_max, mid_split)
constexpr int kSmallMaxMin = 256;
constexpr int kMidSplitMin = 2048;
constexpr int kChunk = 8192;         // larger nodes: (node, projection, sample chunk) items
constexpr int kXcdChunks = 16;       // big nodes of this many chunks or more: XCD-local item layout
constexpr int kXcds = 8;             // XCDs of the device (workgroups are dealt to them round-robin)
constexpr int kSortMax = SOF_SORT_LIMIT;
constexpr int kVcUnit = 256;         // allocation unit of the big-node value cache (floats)

// header counters of the find-splits workspace
enum {
    H_SMALL = 0,   // small node items
    H_DMID,        // mid descriptors
    H_IMID,        // mid items
    H_DSB,         // sort-block descriptors
    H_ISB,         // sort-block items
    H_DBIG,        // big descriptors
    H_IBIGA,       // big (projection, chunk) items
    H_IBIGC,       // big (node, projection) items
    H_SLOTS,       // candidate slots
    H_BIGSLOTS,    // big projection slots (merged range)
    H_DMID2,       // mid descriptors of nodes above kMidSplit samples
    H_IMID2,       // their items
    H_VCACHE,      // projected-value cache of big nodes, in units of kVcUnit floats
    H_Q_MID = 16,  // dequeue counters
    H_Q_SMALL,
    H_Q_SB,
    H_Q_MID2,
    H_Q_BRANGE = 20,   // dequeue counters of the big-node kernels (blocks of per-wave items)
    H_Q_BMERGE,
    H_Q_BHIST,
    H_Q_BSCAN,
    H_ERR = 32,
    H_COUNT = 64
};

struct ProjCSR {
    const int32_t* proj_offsets;
    const int32_t* nz_offsets;
    const int32_t* nz_feature;
    const int8_t* nz_weight;
    int32_t n_proj;
    int64_t n_nz;
    const float* nz_value;   // FP32 weights, or NULL: the integer weights nz_weight
};

// FP32 bits of the weight of nonzero j
__device__ __forceinline__ uint32_t csr_weight_bits(const ProjCSR& P, int64_t j) {
    return P.nz_value ? __float_as_uint(P.nz_value[j]) : __float_as_uint((float)P.nz_weight[j]);
}

// Projections drawn on the fly from a counter-based hash (forest growth):
// node v of the frontier belongs to tree tree_of[v] at position pos_of[v] of
// that tree's frontier at level *level.
struct ProjHash {
    const int32_t* tree_of;
    const int32_t* pos_of;
    const int32_t* level;
    uint64_t seed;
    int32_t k, z;
    int32_t mode, wmode;     // SOF_SAMPLER_*, SOF_WEIGHTS_*
};

struct FindWs {
    int32_t* hdr;
    int4* small_items;    // per small node: (node, s0, n | k << 16, q0)
    int4* desc_mid;
    int4* desc_mid2;
    int4* desc_sb;
    int4* desc_big;       // two int4 per big node
    int4* items_mid;      // two int4 per mid item: (node, slot, group, k), (s0, n, q0, 0)
    int4* items_mid2;
    int2* items_sb;
    int2* items_biga;
    int2* items_bigc;
    void* slots;          // Cand[]
    float2* crange;       // per big item: (min, max) of the chunk
    float2* brange;       // per big slot: (min, max) over the node
    int32_t* phist;       // per big projection slot: [bins][classes] summed over the node's chunks
    float* vcache;        // big nodes: projected values of the range pass, [projection][sample] per node
    double* flnk;         // entropy criterion: k ln k for k = 0 .. cap_flnk - 1
    int64_t cap_small, cap_dmid, cap_imid, cap_dsb, cap_isb, cap_dbig, cap_ibiga, cap_ibigc;
    int64_t cap_slots, cap_bigslots, cap_dmid2, cap_imid2, cap_vcache, cap_flnk;
};

struct FindArgs {
    const void* x;
    int64_t ld;
    const int32_t* y;
    int32_t n_rows, n_features, n_classes, dtype;
    const int32_t* node_offsets;
    const int32_t* sample_idx;
    int64_t n_samples;
    int32_t n_nodes;            // host count, or the capacity when n_nodes_dev is set
    const int32_t* n_nodes_dev; // device count (forest growth), or NULL
    const int32_t* node_bins;
    int32_t bins, sort_threshold;  // sort_threshold already clamped
    int32_t small_max, mid_split;  // wave tile edges (sof_params; 0 there means kSmallMax, kMidSplit)
    int32_t bin_mode;           // SOF_BINS_EQUAL or SOF_BINS_RANDOM
    int32_t criterion;          // SOF_CRIT_GINI or SOF_CRIT_ENTROPY
    uint64_t bin_seed;
    void* out;                  // SplitRec[n_nodes]
    int32_t* hist_out;
    FindWs ws;
};

// Byte layout of the find-splits workspace for the given sizes.
struct FindLayout {
    size_t hdr, small_items, desc_mid, desc_mid2, desc_sb, desc_big, items_mid, items_mid2, items_sb, items_biga,
        items_bigc;
    size_t slots, crange, brange, phist, vcache, flnk, total;
    FindWs caps;
};
// flnk_entries: size of the entropy criterion's k ln k table (0 for Gini)
// vcache = false lays out no projected-value cache (big nodes then re-gather
// their columns in the histogram pass)
FindLayout find_layout(int64_t n_nodes, int64_t n_samples, int64_t n_proj, int64_t max_k, int bins,
                       int classes, int64_t flnk_entries = 0, bool vcache = true);
// table entries for a call: counts reach the largest node's size; capped at
// 2^20 (8 MiB), above which f is computed directly
inline int64_t flnk_entries(int criterion, int64_t max_node_samples) {
    if (criterion != SOF_CRIT_ENTROPY) return 0;
    const int64_t n = max_node_samples + 1;
    return n < (int64_t(1) << 20) ? n : (int64_t(1) << 20);
}
void find_bind(const FindLayout& L, void* ws, FindWs* out);

struct LaunchCfg {
    int n_cu;
    int grid_mid, grid_mid2, grid_small, grid_sort, grid_brange, grid_bhist, grid_bscan, grid_light;
    size_t smem_main, smem_sort;
};

// Streams of one find-splits launch sequence: the caller's stream runs the
// plan; the size classes then run on three streams at once (the caller's and
// the context's two auxiliary streams, forked with `fork` and joined back with
// `join`), and the reduction runs on the caller's stream after the join.
// aux[0] == NULL runs everything on the caller's stream.
struct FindStreams {
    hipStream_t main;
    hipStream_t aux[2];
    hipEvent_t fork;
    hipEvent_t join[2];
};

// Stage timing events (optional): ev[2 s] and ev[2 s + 1] are recorded on the
// stream of stage s before and after it; ev[2 SOF_STAGE_COUNT] and
// ev[2 SOF_STAGE_COUNT + 1] around the whole sequence on the caller's stream.
constexpr int kTimingEvents = 2 * SOF_STAGE_COUNT + 2;

// launchers (return hipError_t)
hipError_t launch_find_csr(const FindArgs& a, const ProjCSR& p, const LaunchCfg& cfg, const FindStreams& st,
                           const hipEvent_t* ev = nullptr);
hipError_t launch_find_hash(const FindArgs& a, const ProjHash& p, const LaunchCfg& cfg, const FindStreams& st,
                            const hipEvent_t* ev = nullptr);
size_t find_smem_main(int bins, int classes, bool random_bins, bool entropy);
size_t find_smem_sort();
// mode: bit 0 random-width bins, bit 1 entropy criterion
hipError_t find_occupancy(int bins, int classes, int mode, int n_cu, LaunchCfg* cfg);

}  // namespace sof
