// k_project.hip -- step 1 alone (paper section 4, step 1: the projected
// feature of every active sample as a sum of weighted columns) and the
// device-side content checks enabled by SOF_CHECK=1.
//
//   k_proj_sizes + k_scan_excl_1blk   output offset of every node (sum n_v k_v)
//   k_pj_plan    (node, group of 4 projections, 8192-sample chunk) items
//   k_project    one block per item, one wave per projection, 16 samples per
//                lane per step with every column's loads issued together
#include <cstring>

#include "sof_device.h"
#include "sof_host.h"
#include "sof_internal.h"

namespace sof {


__device__ __forceinline__ int64_t clampj(int64_t x, int64_t lo, int64_t hi) {
    return x < lo ? lo : (x > hi ? hi : x);
}

__global__ void k_proj_sizes(const int32_t* node_offsets, const int32_t* proj_offsets, int N, int64_t S,
                             int P, int64_t* sizes) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < N; v += gridDim.x * blockDim.x) {
        int64_t a = clampj(node_offsets[v], 0, S), b = clampj(node_offsets[v + 1], a, S);
        int64_t pa = clampj(proj_offsets[v], 0, P), pb = clampj(proj_offsets[v + 1], pa, P);
        sizes[v] = (b - a) * (pb - pa);
    }
}

// exclusive scan of N int64 values in place (one block; a debug-path helper)
__global__ __launch_bounds__(1024) void k_scan_excl_1blk(int64_t* a, int N) {
    extern __shared__ __align__(16) char smem[];
    int64_t* part = (int64_t*)smem;      // 16 wave totals
    int64_t& carry = part[16];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base <= N; base += 1024) {
        const int i = base + tid;
        int64_t x = i < N ? a[i] : 0;
        int64_t incl = x;
        for (int off = 1; off < 64; off <<= 1) {
            int64_t t = __shfl_up(incl, off);
            if (lane >= off) incl += t;
        }
        if (lane == 63) part[w] = incl;
        __syncthreads();
        int64_t before = carry;
        for (int ww = 0; ww < w; ++ww) before += part[ww];
        int64_t tot = carry;
        for (int ww = 0; ww < 16; ++ww) tot += part[ww];
        if (i <= N) a[i] = before + incl - x;
        __syncthreads();
        if (tid == 0) carry = tot;
        __syncthreads();
    }
}

// Work items of the projection: (node, group of kPjGroup projections, chunk
// of kPjChunk samples), one block each, wave w taking projection
// kPjGroup * group + w.  The plan writes them with wave-aggregated
// allocation; a wave writes the items of its nodes together.
constexpr int kPjGroup = 4;          // projections per item (one per wave)
constexpr int kPjChunk = 8192;       // samples per item
constexpr int kPjR = 16;             // samples per lane per step

__global__ __launch_bounds__(256) void k_pj_plan(FindArgs A, ProjCSR P, int32_t* hdr, int4* items,
                                                 int64_t cap) {
    const int N = A.n_nodes;
    const int lane = lane_id();
    for (int v0 = blockIdx.x * 256; v0 < N; v0 += gridDim.x * 256) {
        const int v = v0 + threadIdx.x;
        int cnt = 0, ng = 0, nch = 0;
        if (v < N) {
            const int64_t a = clampj(A.node_offsets[v], 0, A.n_samples);
            const int64_t n = clampj(A.node_offsets[v + 1], a, A.n_samples) - a;
            const int64_t pa = clampj(P.proj_offsets[v], 0, P.n_proj);
            const int k = (int)(clampj(P.proj_offsets[v + 1], pa, P.n_proj) - pa);
            ng = (k + kPjGroup - 1) / kPjGroup;
            nch = (int)((n + kPjChunk - 1) / kPjChunk);
            cnt = ng * nch;
        }
        const int ctr[1] = {0};
        const int c[1] = {cnt};
        int o[1];
        wave_alloc_n<1>(hdr, ctr, c, o);
        uint64_t m = __ballot(cnt > 0);
        while (m) {
            const int src = __builtin_ctzll(m);
            m &= m - 1;
            const int bv = __builtin_amdgcn_readlane(v, src);
            const int bn = __builtin_amdgcn_readlane(cnt, src);
            const int bch = __builtin_amdgcn_readlane(nch, src);
            const int bo = __builtin_amdgcn_readlane(o[0], src);
            for (int t = lane; t < bn; t += kWave)
                if (bo + (int64_t)t < cap) items[bo + t] = make_int4(bv, t / bch, t % bch, 0);
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_project(FindArgs A, ProjCSR P, const int64_t* out_off, float* out,
                                                 int32_t* hdr, const int4* items, int64_t cap) {
    __shared__ int s_item;
    __shared__ int32_t s_lf[kPjGroup][16];
    __shared__ uint32_t s_ls[kPjGroup][16];
    const int w = threadIdx.x >> 6, lane = lane_id();
    const int ni = (int)(hdr[0] < cap ? hdr[0] : cap);
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(&hdr[1], 1);
        __syncthreads();
        const int it = s_item;
        if (it >= ni) break;
        const int4 e = items[it];
        const int v = e.x;
        if (v < 0 || v >= A.n_nodes) continue;
        const int64_t a = clampj(A.node_offsets[v], 0, A.n_samples);
        const int64_t n = clampj(A.node_offsets[v + 1], a, A.n_samples) - a;
        const int64_t pa = clampj(P.proj_offsets[v], 0, P.n_proj);
        const int k = (int)(clampj(P.proj_offsets[v + 1], pa, P.n_proj) - pa);
        const int p = e.y * kPjGroup + w;
        if (p >= k) continue;   // whole wave: no block barrier below
        // stage the wave's projection (lane j: nonzero j)
        const int64_t j0 = clampj(P.nz_offsets[pa + p], 0, P.n_nz);
        int64_t j1 = clampj(P.nz_offsets[pa + p + 1], j0, P.n_nz);
        if (j1 - j0 > SOF_MAX_NNZ) j1 = j0 + SOF_MAX_NNZ;
        const int z = __builtin_amdgcn_readfirstlane((int)(j1 - j0));
        if (lane < z) {
            const uint32_t f = (uint32_t)P.nz_feature[j0 + lane];
            s_lf[w][lane] = f < (uint32_t)A.n_features ? (int)f : 0;
            s_ls[w][lane] = csr_weight_bits(P, j0 + lane);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int64_t c0 = (int64_t)e.z * kPjChunk;
        const int cn = (int)clampj(n - c0, 0, kPjChunk);
        const int32_t* sidx = A.sample_idx + a + c0;
        float* dst = out + out_off[v] + (int64_t)p * n + c0;
        for (int i0 = 0; i0 < cn; i0 += kWave * kPjR) {
            // slots past the chunk's end repeat its last sample (valid
            // addresses, every column's loads issued together) and are not stored
            uint32_t off[kPjR];
#pragma unroll
            for (int r = 0; r < kPjR; ++r) {
                const int i = i0 + r * kWave + lane;
                const uint32_t row = (uint32_t)sidx[i < cn ? i : cn - 1];
                off[r] = (row < (uint32_t)A.n_rows ? row : 0u) * (uint32_t)sizeof(T);
            }
            float val[kPjR];
#pragma unroll
            for (int r = 0; r < kPjR; ++r) val[r] = 0.f;
            for (int j = 0; j < z; ++j) {
                const int f = __builtin_amdgcn_readfirstlane(s_lf[w][j]);
                const uint32_t sg = __builtin_amdgcn_readfirstlane(s_ls[w][j]);
                const T* col = (const T*)A.x + (int64_t)f * A.ld;
                float x[kPjR];
#pragma unroll
                for (int r = 0; r < kPjR; ++r) x[r] = ldx((const T*)((const char*)col + off[r]), 0);
#pragma unroll
                for (int r = 0; r < kPjR; ++r) val[r] = __fadd_rn(val[r], weighted_term(x[r], sg));
            }
#pragma unroll
            for (int r = 0; r < kPjR; ++r) {
                const int i = i0 + r * kWave + lane;
                if (i < cn) dst[i] = val[r];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// content checks

enum {
    CK_NODE_OFFSETS = 1, CK_NODE_SIZE = 2, CK_SAMPLE = 4, CK_PROJ_OFFSETS = 8, CK_PROJ_COUNT = 16,
    CK_NZ_OFFSETS = 32, CK_NZ_COUNT = 64, CK_FEATURE = 128, CK_DISTINCT = 256, CK_WEIGHT = 512,
    CK_LABEL = 1024, CK_BINS = 2048
};

__global__ void k_check(sof_data D, sof_frontier F, sof_proj P, sof_params Q, int32_t* flag) {
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t gs = (int64_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (int64_t v = gid; v <= F.n_nodes; v += gs) {
        int32_t o = F.node_offsets[v];
        if (v == 0 && o != 0) bad |= CK_NODE_OFFSETS;
        if (v == F.n_nodes && o != F.n_samples) bad |= CK_NODE_OFFSETS;
        if (v < F.n_nodes) {
            int32_t o1 = F.node_offsets[v + 1];
            if (o1 < o) bad |= CK_NODE_OFFSETS;
            if (o1 - o > F.max_node_samples) bad |= CK_NODE_SIZE;
            int32_t p0 = P.proj_offsets[v], p1 = P.proj_offsets[v + 1];
            if (p1 < p0) bad |= CK_PROJ_OFFSETS;
            if (p1 - p0 > P.max_proj_per_node) bad |= CK_PROJ_COUNT;
            if (Q.node_bins) {
                int b = Q.node_bins[v];
                if (b < 2 || b > Q.bins) bad |= CK_BINS;
            }
        }
        int32_t po = P.proj_offsets[v];
        if (v == 0 && po != 0) bad |= CK_PROJ_OFFSETS;
        if (v == F.n_nodes && po != P.n_proj) bad |= CK_PROJ_OFFSETS;
    }
    for (int64_t i = gid; i < F.n_samples; i += gs)
        if ((uint32_t)F.sample_idx[i] >= (uint32_t)D.n_rows) bad |= CK_SAMPLE;
    for (int64_t r = gid; r < D.n_rows; r += gs)
        if ((uint32_t)D.y[r] >= (uint32_t)D.n_classes) bad |= CK_LABEL;
    for (int64_t q = gid; q <= P.n_proj; q += gs) {
        int32_t o = P.nz_offsets[q];
        if (q == 0 && o != 0) bad |= CK_NZ_OFFSETS;
        if (q == P.n_proj && o != P.n_nz) bad |= CK_NZ_OFFSETS;
        if (q < P.n_proj) {
            int32_t o1 = P.nz_offsets[q + 1];
            if (o1 < o) bad |= CK_NZ_OFFSETS;
            if (o1 - o > SOF_MAX_NNZ || o1 - o < 0) bad |= CK_NZ_COUNT;
            else if (o >= 0 && o1 <= P.n_nz)
                for (int32_t j = o; j < o1; ++j) {
                    int32_t f = P.nz_feature[j];
                    if ((uint32_t)f >= (uint32_t)D.n_features) bad |= CK_FEATURE;
                    if (P.nz_value && !__builtin_isfinite(P.nz_value[j])) bad |= CK_WEIGHT;
                    for (int32_t j2 = o; j2 < j; ++j2)
                        if (P.nz_feature[j2] == f) bad |= CK_DISTINCT;
                }
        }
    }
    if (bad) atomicOr(flag, bad);
}

// Workspace: the output offsets (N + 1 int64), two counters, the items.  A
// node has ceil(k/4) ceil(n/8192) items, at most (k + 3)(n + 8191) / 32768;
// summed over nodes (k <= 1024) that is below S/32 + 3S/32768 + P/4 + N,
// which the capacity covers.
static int64_t pj_items_cap(int64_t n_nodes, int64_t n_samples, int64_t n_proj) {
    return n_proj / 4 + n_nodes + n_samples / kPjChunk + (1024 / kPjGroup + 1) * (n_samples / kPjChunk + 1) + 1;
}
size_t project_workspace(int64_t n_nodes, int64_t n_samples, int64_t n_proj) {
    size_t o = ((size_t)(n_nodes + 1) * sizeof(int64_t) + 255) & ~(size_t)255;
    o += 256;   // counters
    o += (size_t)pj_items_cap(n_nodes, n_samples, n_proj) * sizeof(int4);
    return (o + 255) & ~(size_t)255;
}

int device_check(sof_ctx* ctx, const sof_data* data, const sof_frontier* fr, const sof_proj* proj,
                 const sof_params* params, hipStream_t s) {
    int32_t* flag = nullptr;
    hipError_t e = hipMalloc(&flag, sizeof(int32_t));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc (SOF_CHECK flag)");
    int32_t zero = 0, got = 0;
    e = hipMemcpyAsync(flag, &zero, sizeof(zero), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_check, dim3(ctx->n_cu * 4), dim3(256), 0, s, *data, *fr, *proj, *params, flag);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&got, flag, sizeof(got), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(flag);
    if (e != hipSuccess) return hip_fail(e, "SOF_CHECK kernel");
    if (got) {
        std::string what;
        const char* names[] = {"node_offsets", "node size above max_node_samples", "sample_idx out of range",
                               "proj_offsets", "projections per node above max_proj_per_node",
                               "nz_offsets", "nonzeros per projection above 16", "feature id out of range",
                               "repeated feature in a projection", "weight not finite", "label out of range",
                               "node_bins out of range"};
        for (int b = 0; b < 12; ++b)
            if (got & (1 << b)) { if (!what.empty()) what += ", "; what += names[b]; }
        return fail(SOF_ERR_DEVICE, "SOF_CHECK: %s", what.c_str());
    }
    return SOF_OK;
}

__global__ void k_pj_reset(int32_t* hdr) {
    if (threadIdx.x < 2) hdr[threadIdx.x] = 0;
}

hipError_t launch_project(const FindArgs& a, const ProjCSR& p, float* out, void* ws, int n_cu,
                          hipStream_t s) {
    int64_t* off = (int64_t*)ws;
    const int N = a.n_nodes;
    char* b = (char*)ws + (((size_t)(N + 1) * sizeof(int64_t) + 255) & ~(size_t)255);
    int32_t* hdr = (int32_t*)b;
    int4* items = (int4*)(b + 256);
    const int64_t cap = pj_items_cap(N, a.n_samples, p.n_proj);
    int g = (N + 255) / 256;
    if (g > 4 * n_cu) g = 4 * n_cu;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_proj_sizes, dim3(g), dim3(256), 0, s, a.node_offsets, p.proj_offsets, N, a.n_samples,
                       p.n_proj, off);
    hipLaunchKernelGGL(k_scan_excl_1blk, dim3(1), dim3(1024), 17 * sizeof(int64_t), s, off, N);
    if (p.n_proj > 0) {
        hipLaunchKernelGGL(k_pj_reset, dim3(1), dim3(64), 0, s, hdr);
        hipLaunchKernelGGL(k_pj_plan, dim3(g), dim3(256), 0, s, a, p, hdr, items, cap);
        if (a.dtype == SOF_F16)
            hipLaunchKernelGGL(k_project<_Float16>, dim3(n_cu * 8), dim3(256), 0, s, a, p, (const int64_t*)off, out,
                               hdr, (const int4*)items, cap);
        else
            hipLaunchKernelGGL(k_project<float>, dim3(n_cu * 8), dim3(256), 0, s, a, p, (const int64_t*)off, out,
                               hdr, (const int4*)items, cap);
    }
    return hipGetLastError();
}

}  // namespace sof

using namespace sof;

extern "C" int sof_project(sof_ctx* ctx, const sof_data* data, const sof_frontier* fr, const sof_proj* proj,
                           float* out, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx) return fail(SOF_ERR_INVALID_ARG, "ctx is NULL");
    int rc;
    if ((rc = check_data(data)) || (rc = check_frontier(fr)) || (rc = check_proj(proj, data))) return rc;
    if (proj->n_proj > 0 && fr->n_samples > 0 && !out) return fail(SOF_ERR_INVALID_ARG, "out is NULL");
    if ((rc = check_ws_public(ws, ws_bytes, project_workspace(fr->n_nodes, fr->n_samples, proj->n_proj)))) return rc;
    if (fr->n_nodes == 0) return SOF_OK;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    sof_params q{nullptr, 256, 0};
    FindArgs a;
    fill_find_args(data, fr, &q, nullptr, nullptr, &a);
    ProjCSR p{proj->proj_offsets, proj->nz_offsets, proj->nz_feature, proj->nz_weight, proj->n_proj, proj->n_nz,
              proj->nz_value};
    e = launch_project(a, p, out, ws, ctx->n_cu, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "project launch");
    return SOF_OK;
}
