// sof_host.h -- host-side internals of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "sof.h"
#include "sof_internal.h"

struct sof_ctx {
    int device = 0;
    int n_cu = 0;
    size_t lds_per_block = 0;
    bool check = false;
    std::mutex mu;
    std::map<std::pair<int, int>, sof::LaunchCfg> cfg;   // key (4 * bins + mode, classes)
    bool timing = false;                             // benchmark instrumentation
    bool timing_serial = false;                      // ... with the size classes serialised
    bool timing_whole = false;                       // ... around the whole call only
    // one event set per recorded call; in tev_whole only the whole call's
    // pair exists (the stage entries are null)
    std::vector<std::array<hipEvent_t, sof::kTimingEvents>> tev, tev_whole;
    size_t tev_used = 0;
    void* scratch = nullptr;   // device address of this device's static scratch array
    // the find-splits and partition sequences fork their size classes onto
    // two auxiliary streams (default priority) and join them back with these
    // events;
    // launch_mu keeps two host threads from interleaving their forks
    hipStream_t aux[2] = {nullptr, nullptr};
    hipEvent_t fork = nullptr;
    hipEvent_t join[2] = {nullptr, nullptr};
    std::mutex launch_mu;
};

namespace sof {
// the context's streams around a launch on the caller's stream s
inline FindStreams find_streams(sof_ctx* ctx, hipStream_t s) {
    if (ctx->timing && ctx->timing_serial) return FindStreams{s, {nullptr, nullptr}, nullptr, {nullptr, nullptr}};
    return FindStreams{s, {ctx->aux[0], ctx->aux[1]}, ctx->fork, {ctx->join[0], ctx->join[1]}};
}
}  // namespace sof

namespace sof {

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

int check_data(const sof_data* d);
int check_frontier(const sof_frontier* f);
int check_proj(const sof_proj* p, const sof_data* d);
int check_params(const sof_params* q);
int check_ws_public(void* ws, size_t ws_bytes, size_t need);
int clamp_threshold(int t);

// mode: bit 0 random-width bins, bit 1 entropy criterion
int launch_cfg(sof_ctx* ctx, int bins, int classes, int mode, LaunchCfg* cfg);
int fill_find_args(const sof_data* data, const sof_frontier* fr, const sof_params* params,
                   sof_split* out, int32_t* hist_out, FindArgs* a);

// partition
struct PartArgs {
    const void* x;
    int64_t ld;
    int32_t n_rows, n_features, dtype;
    const int32_t* node_offsets;
    const int32_t* sample_idx;
    int64_t n_samples;
    int32_t n_nodes;
    const int32_t* n_nodes_dev;
    const int32_t* node_bins;
    int32_t bins;
    const void* splits;       // SplitRec[n_nodes]
    int32_t* out_idx;
    int32_t* child_offsets;
    // workspace
    int32_t* hdr;             // counters
    int4* big_items;          // (node, chunk, chunk count, first item of the node)
    int32_t* chunk_left;      // left count per chunk item
    int64_t* chunk_pre;       // exclusive prefix of chunk_left over all chunk items
    uint64_t* pred_bits;      // one bit per sample of every chunk item
    int64_t cap_items;
};
size_t part_workspace(int64_t n_nodes, int64_t n_samples);
void part_bind(int64_t n_nodes, int64_t n_samples, void* ws, PartArgs* a);
hipError_t launch_partition_csr(const PartArgs& a, const ProjCSR& p, int n_cu, const FindStreams& st);
hipError_t launch_partition_hash(const PartArgs& a, const ProjHash& p, int n_cu, const FindStreams& st);

// projection only
size_t project_workspace(int64_t n_nodes, int64_t n_samples, int64_t n_proj);
hipError_t launch_project(const FindArgs& a, const ProjCSR& p, float* out, void* ws, int n_cu,
                          hipStream_t s);

// content checks (SOF_CHECK=1)
int device_check(sof_ctx* ctx, const sof_data* data, const sof_frontier* fr, const sof_proj* proj,
                 const sof_params* params, hipStream_t s);

}  // namespace sof
