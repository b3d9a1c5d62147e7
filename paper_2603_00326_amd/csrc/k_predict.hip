// k_predict.hip -- prediction with grown trees: every tree votes the label of
// the leaf a row reaches, the class with most votes wins (lowest on ties).
// The forests the paper trains (section 2) are grown to purity; an internal
// node sends a row left when its rule holds on the row's projection v (the
// node's own features and FP32 weights, one rounding per product and per add
// in feature order from +0):
// equal-width bins bin(v) <= bin, sort splits v <= threshold, random-width
// bins v < threshold.
//
// One thread per query row walks the trees in turn.  A node record (200
// bytes, 8-byte aligned) is read as twenty-four 8-byte loads issued together
// (header, feature ids, weights; not the gain), then the node's column
// gathers, so a level costs two dependent round trips.  Every index taken from a record is
// checked, and a walk stops after 130 steps (a tree is at most 65 levels
// deep), so damaged records cannot run away.
#include <hip/hip_runtime.h>

#include "sof.h"
#include "sof_device.h"
#include "sof_host.h"
#include "sof_internal.h"

namespace sof {

static_assert(sizeof(sof_tree_node) == 200, "sof_tree_node layout");

struct PredArgs {
    const void* x;
    int64_t ld;
    int32_t n_rows, n_features, n_classes, n_trees;
    const sof_tree_node* nodes;
    int64_t n_nodes;
    const int32_t* roots;
    int32_t* votes;   // n_rows * n_classes, or NULL
    int32_t* pred;    // n_rows
};

constexpr int kPredictSteps = 130;

constexpr int kRecWords = 24;

// q: the record as int2 words (8k = byte offset): 0 tree, depth; 1 parent,
// left; 2 right, n_samples; 3 label, is_leaf; 4 kind, bin; 5 threshold, lo;
// 6 scale, n_bins; 7 nnz, pad; 8..15 feature ids; 16..23 weights (FP32 x 16)
template <typename T>
__device__ __forceinline__ float node_value(const PredArgs& a, const int2* q, int nnz, int32_t row) {
    const int32_t f[16] = {q[8].x, q[8].y, q[9].x, q[9].y, q[10].x, q[10].y, q[11].x, q[11].y,
                           q[12].x, q[12].y, q[13].x, q[13].y, q[14].x, q[14].y, q[15].x, q[15].y};
    const int32_t wb[16] = {q[16].x, q[16].y, q[17].x, q[17].y, q[18].x, q[18].y, q[19].x, q[19].y,
                            q[20].x, q[20].y, q[21].x, q[21].y, q[22].x, q[22].y, q[23].x, q[23].y};
    float acc = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (j >= nnz) break;
        const uint32_t fj = (uint32_t)f[j] < (uint32_t)a.n_features ? (uint32_t)f[j] : 0u;
        const float x = ldx((const T*)a.x + (int64_t)fj * a.ld, row);
        acc = __fadd_rn(acc, weighted_term(x, (uint32_t)wb[j]));
    }
    return acc;
}

template <typename T>
__global__ __launch_bounds__(256) void k_predict(PredArgs a) {
    const int C = a.n_classes;
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < a.n_rows; r += (int64_t)gridDim.x * 256) {
        uint32_t cnt[SOF_MAX_CLASSES];
#pragma unroll
        for (int c = 0; c < SOF_MAX_CLASSES; ++c) cnt[c] = 0;
        for (int t = 0; t < a.n_trees; ++t) {
            int64_t i = a.roots[t];
            int label = -1;
            for (int step = 0; step < kPredictSteps; ++step) {
                if (i < 0 || i >= a.n_nodes) break;
                const int2* rec = (const int2*)(a.nodes + i);
                int2 q[kRecWords];
#pragma unroll
                for (int u = 0; u < kRecWords; ++u) q[u] = rec[u];
                if (q[3].y) {
                    label = q[3].x;
                    break;
                }
                const int kind = q[4].x;
                const int nnz = q[7].x < 0 ? 0 : (q[7].x > SOF_MAX_NNZ ? SOF_MAX_NNZ : q[7].x);
                const float v = node_value<T>(a, q, nnz, (int32_t)r);
                const float thr = __int_as_float(q[5].x);
                bool left;
                if (kind == SOF_SPLIT_HIST) {
                    const int nb = q[6].y < SOF_MIN_BINS ? SOF_MIN_BINS : (q[6].y > SOF_MAX_BINS ? SOF_MAX_BINS : q[6].y);
                    left = bin_index(v, __int_as_float(q[5].y), __int_as_float(q[6].x), nb) <= q[4].y;
                } else if (kind == SOF_SPLIT_RHIST) {
                    left = v < thr;
                } else {
                    left = v <= thr;
                }
                i = left ? q[1].y : q[2].x;
            }
#pragma unroll
            for (int c = 0; c < SOF_MAX_CLASSES; ++c) cnt[c] += (label == c) ? 1u : 0u;
        }
        int best = 0;
        uint32_t bv = cnt[0];
#pragma unroll
        for (int c = 1; c < SOF_MAX_CLASSES; ++c)
            if (c < C && cnt[c] > bv) { bv = cnt[c]; best = c; }
        a.pred[r] = best;
        if (a.votes) {
#pragma unroll
            for (int c = 0; c < SOF_MAX_CLASSES; ++c)
                if (c < C) a.votes[r * C + c] = (int32_t)cnt[c];
        }
    }
}

}  // namespace sof

// ---------------------------------------------------------------------------
// C ABI

using namespace sof;

extern "C" int sof_predict(sof_ctx* ctx, const sof_data* data, const sof_tree_node* nodes, int64_t n_nodes,
                           const int32_t* roots, int32_t n_trees, int32_t* votes, int32_t* pred, void* stream) {
    if (!ctx) return fail(SOF_ERR_INVALID_ARG, "ctx is NULL");
    if (!data || !data->x) return fail(SOF_ERR_INVALID_ARG, "data or data->x is NULL");
    if (data->dtype != SOF_F32 && data->dtype != SOF_F16)
        return fail(SOF_ERR_UNSUPPORTED, "dtype %d (expected SOF_F32 or SOF_F16)", data->dtype);
    if (data->n_classes < 2 || data->n_classes > SOF_MAX_CLASSES)
        return fail(SOF_ERR_UNSUPPORTED, "n_classes %d outside [2, %d]", data->n_classes, SOF_MAX_CLASSES);
    if (data->n_rows < 0 || data->n_features < 1 || data->ld < data->n_rows)
        return fail(SOF_ERR_INVALID_ARG, "n_rows %d, n_features %d, ld %lld", data->n_rows, data->n_features,
                    (long long)data->ld);
    if (n_trees < 1 || n_nodes < 1 || !nodes || !roots)
        return fail(SOF_ERR_INVALID_ARG, "need nodes, roots and at least one tree");
    if (data->n_rows > 0 && !pred) return fail(SOF_ERR_INVALID_ARG, "pred is NULL");
    if (data->n_rows == 0) return SOF_OK;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    PredArgs a{data->x, data->ld, data->n_rows, data->n_features, data->n_classes, n_trees, nodes, n_nodes,
               roots, votes, pred};
    int64_t blocks = ((int64_t)data->n_rows + 255) / 256;
    const int64_t cap = (int64_t)ctx->n_cu * 16;
    if (blocks > cap) blocks = cap;
    if (data->dtype == SOF_F16)
        hipLaunchKernelGGL(k_predict<_Float16>, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, a);
    else
        hipLaunchKernelGGL(k_predict<float>, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "predict launch");
    return SOF_OK;
}
