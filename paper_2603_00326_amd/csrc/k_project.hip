// k_project.hip -- step 1 alone (paper section 4, step 1: the projected
// feature of every active sample as a sum of weighted columns) and the
// device-side content checks enabled by SOF_CHECK=1.
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

template <typename T>
__global__ __launch_bounds__(256) void k_project(FindArgs A, ProjCSR P, const int64_t* out_off, float* out) {
    extern __shared__ __align__(16) char smem[];
    int32_t* lf = (int32_t*)smem;        // staged nonzeros
    uint32_t* ls = (uint32_t*)(lf + 16);
    int& s_z = *(int*)(ls + 16);
    int& s_v = *(&s_z + 1);
    const int N = A.n_nodes;
    for (int q = blockIdx.x; q < P.n_proj; q += gridDim.x) {
        if (threadIdx.x == 0) {
            // node owning projection q: last v with proj_offsets[v] <= q
            int lo = 0, hi = N;
            while (hi - lo > 1) {
                int mid = (lo + hi) >> 1;
                if (P.proj_offsets[mid] <= q) lo = mid; else hi = mid;
            }
            s_v = lo;
            int64_t j0 = clampj(P.nz_offsets[q], 0, P.n_nz), j1 = clampj(P.nz_offsets[q + 1], j0, P.n_nz);
            if (j1 - j0 > SOF_MAX_NNZ) j1 = j0 + SOF_MAX_NNZ;
            s_z = (int)(j1 - j0);
            for (int j = 0; j < s_z; ++j) {
                uint32_t f = (uint32_t)P.nz_feature[j0 + j];
                lf[j] = f < (uint32_t)A.n_features ? (int)f : 0;
                ls[j] = csr_weight_bits(P, j0 + j);
            }
        }
        __syncthreads();
        const int v = s_v, z = s_z;
        const int64_t a = clampj(A.node_offsets[v], 0, A.n_samples);
        const int64_t n = clampj(A.node_offsets[v + 1], a, A.n_samples) - a;
        const int p = q - (int)clampj(P.proj_offsets[v], 0, P.n_proj);
        const int kv = (int)(clampj(P.proj_offsets[v + 1], 0, P.n_proj) - clampj(P.proj_offsets[v], 0, P.n_proj));
        if (p < 0 || p >= kv) { __syncthreads(); continue; }
        float* dst = out + out_off[v] + (int64_t)p * n;
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            uint32_t r = (uint32_t)A.sample_idx[a + i];
            const int row = r < (uint32_t)A.n_rows ? (int)r : 0;
            float acc = 0.f;
            for (int j = 0; j < z; ++j) {
                const T* col = (const T*)A.x + (int64_t)lf[j] * A.ld;
                acc = __fadd_rn(acc, weighted_term(ldx(col, row), ls[j]));
            }
            dst[i] = acc;
        }
        __syncthreads();
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

size_t project_workspace(int64_t n_nodes) { return ((size_t)(n_nodes + 1) * sizeof(int64_t) + 255) & ~(size_t)255; }

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

hipError_t launch_project(const FindArgs& a, const ProjCSR& p, float* out, void* ws, int n_cu,
                          hipStream_t s) {
    int64_t* off = (int64_t*)ws;
    const int N = a.n_nodes;
    int g = (N + 255) / 256;
    if (g > 4 * n_cu) g = 4 * n_cu;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_proj_sizes, dim3(g), dim3(256), 0, s, a.node_offsets, p.proj_offsets, N, a.n_samples,
                       p.n_proj, off);
    hipLaunchKernelGGL(k_scan_excl_1blk, dim3(1), dim3(1024), 17 * sizeof(int64_t), s, off, N);
    if (p.n_proj > 0) {
        if (a.dtype == SOF_F16)
            hipLaunchKernelGGL(k_project<_Float16>, dim3(n_cu * 8), dim3(256), 256, s, a, p, (const int64_t*)off, out);
        else
            hipLaunchKernelGGL(k_project<float>, dim3(n_cu * 8), dim3(256), 256, s, a, p, (const int64_t*)off, out);
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
    if ((rc = check_ws_public(ws, ws_bytes, project_workspace(fr->n_nodes)))) return rc;
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
