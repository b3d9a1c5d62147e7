// sof_api.hip -- host side of the C ABI: argument validation (runs without a
// GPU), workspace layout, context and launch configuration.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "sof.h"
#include "sof_internal.h"
#include "sof_host.h"

using namespace sof;

// ---------------------------------------------------------------------------
// errors

static thread_local std::string g_err;

int sof::fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int sof::hip_fail(hipError_t e, const char* what) {
    return fail(SOF_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

extern "C" const char* sof_last_error(void) { return g_err.c_str(); }
extern "C" const char* sof_version(void) { return "sof 0.1 gfx950"; }

// ---------------------------------------------------------------------------
// static scratch of sof_find_splits_noalloc
//
// One array per device, loaded with the code object and held until the
// process ends.  In host code its name is only a stand-in for the device
// symbol: the device address comes from hipGetSymbolAddress, taken once per
// device (sof_create) with that device current, and only that address is
// passed to kernels.

static __device__ __align__(256) unsigned char scratch[SOF_STATIC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_ptr;   // device -> address of its scratch

static int scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return SOF_OK;
    }
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress (static scratch)");
    if (!ptr) return fail(SOF_ERR_HIP, "hipGetSymbolAddress returned NULL for the static scratch");
    g_scratch_ptr[device] = ptr;
    *out = ptr;
    return SOF_OK;
}

// ---------------------------------------------------------------------------
// context

extern "C" int sof_create(int device, sof_ctx** out) {
    if (!out) return fail(SOF_ERR_INVALID_ARG, "sof_create: out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count)
        return fail(SOF_ERR_INVALID_ARG, "sof_create: device %d of %d", device, count);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(SOF_ERR_UNSUPPORTED, "sof_create: device is %s, this library is built for gfx950",
                    prop.gcnArchName);
    void* sp = nullptr;
    int rc = scratch_address(device, &sp);
    if (rc) return rc;
    sof_ctx* c = new sof_ctx();
    c->device = device;
    c->scratch = sp;
    c->n_cu = prop.multiProcessorCount;
    c->lds_per_block = (size_t)prop.sharedMemPerBlock;
    const char* chk = getenv("SOF_CHECK");
    c->check = chk && chk[0] == '1';
    int prev = 0;
    e = hipGetDevice(&prev);
    if (e == hipSuccess && prev != device) e = hipSetDevice(device);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&c->aux[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&c->join[i], hipEventDisableTiming);
    if (prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        sof_destroy(c);
        return hip_fail(e, "sof_create: streams and events");
    }
    *out = c;
    return SOF_OK;
}

extern "C" int sof_destroy(sof_ctx* ctx) {
    if (ctx) {
        for (auto* pool : {&ctx->tev, &ctx->tev_whole})
            for (auto& a : *pool)
                for (hipEvent_t e : a)
                    if (e) (void)hipEventDestroy(e);
        for (int i = 0; i < 2; ++i) {
            if (ctx->aux[i]) (void)hipStreamDestroy(ctx->aux[i]);
            if (ctx->join[i]) (void)hipEventDestroy(ctx->join[i]);
        }
        if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    }
    delete ctx;
    return SOF_OK;
}

extern "C" int sof_timing_enable(sof_ctx* ctx, int enable) {
    if (!ctx) return fail(SOF_ERR_INVALID_ARG, "ctx is NULL");
    ctx->timing = enable != 0;
    ctx->timing_serial = enable == 2;
    ctx->timing_whole = enable == 3;
    ctx->tev_used = 0;
    return SOF_OK;
}

extern "C" int sof_timing_read(sof_ctx* ctx, float* ms, int32_t* calls) {
    if (!ctx || !ms || !calls) return fail(SOF_ERR_INVALID_ARG, "NULL argument");
    for (int i = 0; i <= SOF_STAGE_COUNT; ++i) ms[i] = 0.f;
    auto& pool = ctx->timing_whole ? ctx->tev_whole : ctx->tev;
    for (size_t c = 0; c < ctx->tev_used && c < pool.size(); ++c) {
        auto& e = pool[c];
        hipError_t r = hipEventSynchronize(e[kTimingEvents - 1]);
        if (r != hipSuccess) return hip_fail(r, "hipEventSynchronize");
        for (int i = 0; i <= SOF_STAGE_COUNT; ++i) {
            if (!e[2 * i] || !e[2 * i + 1]) continue;
            float t = 0.f;
            r = hipEventElapsedTime(&t, e[2 * i], e[2 * i + 1]);
            if (r != hipSuccess) return hip_fail(r, "hipEventElapsedTime");
            ms[i] += t;
        }
    }
    *calls = (int32_t)ctx->tev_used;
    ctx->tev_used = 0;
    return SOF_OK;
}

// next event set for an instrumented call (allocates events on first use)
static const hipEvent_t* timing_events(sof_ctx* ctx) {
    if (!ctx->timing) return nullptr;
    auto& pool = ctx->timing_whole ? ctx->tev_whole : ctx->tev;
    if (ctx->tev_used == pool.size()) {
        std::array<hipEvent_t, kTimingEvents> a;
        for (int i = 0; i < kTimingEvents; ++i) {
            a[i] = nullptr;
            if (ctx->timing_whole && i < 2 * SOF_STAGE_COUNT) continue;
            if (hipEventCreate(&a[i]) != hipSuccess) {
                for (int j = 0; j < i; ++j)
                    if (a[j]) (void)hipEventDestroy(a[j]);
                return nullptr;
            }
        }
        pool.push_back(a);
    }
    return pool[ctx->tev_used++].data();
}

int sof::launch_cfg(sof_ctx* ctx, int bins, int classes, int mode, LaunchCfg* cfg) {
    std::lock_guard<std::mutex> g(ctx->mu);
    auto key = std::make_pair(4 * bins + (mode & 3), classes);
    auto it = ctx->cfg.find(key);
    if (it != ctx->cfg.end()) {
        *cfg = it->second;
        return SOF_OK;
    }
    LaunchCfg c;
    hipError_t e = find_occupancy(bins, classes, mode, ctx->n_cu, &c);
    if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    if (c.smem_main > ctx->lds_per_block || c.smem_sort > ctx->lds_per_block)
        return fail(SOF_ERR_UNSUPPORTED, "LDS need %zu/%zu bytes exceeds %zu per block", c.smem_main,
                    c.smem_sort, ctx->lds_per_block);
    ctx->cfg[key] = c;
    *cfg = c;
    return SOF_OK;
}

// ---------------------------------------------------------------------------
// validation (host only)

int sof::check_data(const sof_data* d) {
    if (!d) return fail(SOF_ERR_INVALID_ARG, "data is NULL");
    if (d->dtype != SOF_F32 && d->dtype != SOF_F16)
        return fail(SOF_ERR_UNSUPPORTED, "dtype %d (expected SOF_F32 or SOF_F16)", d->dtype);
    if (d->n_classes < 2 || d->n_classes > SOF_MAX_CLASSES)
        return fail(SOF_ERR_UNSUPPORTED, "n_classes %d outside [2, %d]", d->n_classes, SOF_MAX_CLASSES);
    if (d->n_rows < 1 || d->n_features < 1)
        return fail(SOF_ERR_INVALID_ARG, "n_rows %d and n_features %d must be >= 1", d->n_rows,
                    d->n_features);
    if (d->ld < d->n_rows) return fail(SOF_ERR_INVALID_ARG, "ld %lld < n_rows %d", (long long)d->ld, d->n_rows);
    if (d->n_rows > (1 << 30))
        return fail(SOF_ERR_OVERFLOW, "n_rows %d above 2^30", d->n_rows);
    if (!d->x || !d->y) return fail(SOF_ERR_INVALID_ARG, "data->x or data->y is NULL");
    return SOF_OK;
}

int sof::check_frontier(const sof_frontier* f) {
    if (!f) return fail(SOF_ERR_INVALID_ARG, "frontier is NULL");
    if (f->n_nodes < 0) return fail(SOF_ERR_INVALID_ARG, "n_nodes %d < 0", f->n_nodes);
    if (f->n_samples < 0) return fail(SOF_ERR_INVALID_ARG, "n_samples < 0");
    if (f->n_samples > 0x7fffffffLL)
        return fail(SOF_ERR_OVERFLOW, "n_samples %lld above 2^31-1", (long long)f->n_samples);
    if (f->max_node_samples < 0) return fail(SOF_ERR_INVALID_ARG, "max_node_samples < 0");
    if (f->max_node_samples > SOF_MAX_NODE_SAMPLES)
        return fail(SOF_ERR_OVERFLOW, "max_node_samples %d above 2^24", f->max_node_samples);
    if (f->max_node_samples > f->n_samples)
        return fail(SOF_ERR_INVALID_ARG, "max_node_samples %d above n_samples %lld", f->max_node_samples,
                    (long long)f->n_samples);
    if (!f->node_offsets) return fail(SOF_ERR_INVALID_ARG, "node_offsets is NULL");
    if (f->n_samples > 0 && !f->sample_idx) return fail(SOF_ERR_INVALID_ARG, "sample_idx is NULL");
    return SOF_OK;
}

int sof::check_proj(const sof_proj* p, const sof_data* d) {
    if (!p) return fail(SOF_ERR_INVALID_ARG, "proj is NULL");
    if (p->n_proj < 0 || p->n_nz < 0) return fail(SOF_ERR_INVALID_ARG, "n_proj or n_nz < 0");
    if (p->n_nz > 0x7fffffffLL) return fail(SOF_ERR_OVERFLOW, "n_nz above 2^31-1");
    if (p->max_proj_per_node < 0 || p->max_proj_per_node > 1024)
        return fail(SOF_ERR_INVALID_ARG, "max_proj_per_node %d outside [0, 1024]", p->max_proj_per_node);
    if (p->max_proj_per_node > p->n_proj)
        return fail(SOF_ERR_INVALID_ARG, "max_proj_per_node %d above n_proj %d", p->max_proj_per_node,
                    p->n_proj);
    if (!p->proj_offsets || !p->nz_offsets) return fail(SOF_ERR_INVALID_ARG, "proj offsets NULL");
    if (p->n_nz > 0 && (!p->nz_feature || (!p->nz_weight && !p->nz_value)))
        return fail(SOF_ERR_INVALID_ARG, "nz_feature is NULL, or both nz_weight and nz_value are");
    (void)d;
    return SOF_OK;
}

int sof::check_params(const sof_params* q) {
    if (!q) return fail(SOF_ERR_INVALID_ARG, "params is NULL");
    if (q->bins < SOF_MIN_BINS || q->bins > SOF_MAX_BINS)
        return fail(SOF_ERR_UNSUPPORTED, "bins %d outside [2, 256]", q->bins);
    if (q->sort_threshold < 0) return fail(SOF_ERR_INVALID_ARG, "sort_threshold < 0");
    if (q->bin_mode != SOF_BINS_EQUAL && q->bin_mode != SOF_BINS_RANDOM)
        return fail(SOF_ERR_UNSUPPORTED, "bin_mode %d (expected SOF_BINS_EQUAL or SOF_BINS_RANDOM)", q->bin_mode);
    if (q->criterion != SOF_CRIT_GINI && q->criterion != SOF_CRIT_ENTROPY)
        return fail(SOF_ERR_UNSUPPORTED, "criterion %d (expected SOF_CRIT_GINI or SOF_CRIT_ENTROPY)", q->criterion);
    if (q->small_max != 0 && (q->small_max < kSmallMaxMin || q->small_max > kSmallMax))
        return fail(SOF_ERR_INVALID_ARG, "small_max %d outside [%d, %d] (0: %d)", q->small_max, kSmallMaxMin,
                    kSmallMax, kSmallMax);
    if (q->mid_split != 0 && (q->mid_split < kMidSplitMin || q->mid_split > kMidSplit))
        return fail(SOF_ERR_INVALID_ARG, "mid_split %d outside [%d, %d] (0: %d)", q->mid_split, kMidSplitMin,
                    kMidSplit, kMidSplit);
    return SOF_OK;
}

int sof::clamp_threshold(int t) { return t > SOF_SORT_LIMIT + 1 ? SOF_SORT_LIMIT + 1 : t; }

// ---------------------------------------------------------------------------
// workspace layout

static size_t align_up(size_t x) { return (x + SOF_WORKSPACE_ALIGN - 1) & ~(size_t)(SOF_WORKSPACE_ALIGN - 1); }
static int64_t mn(int64_t a, int64_t b) { return a < b ? a : b; }

FindLayout sof::find_layout(int64_t N, int64_t S, int64_t P, int64_t K, int bins, int classes,
                            int64_t flnk_entries, bool vcache) {
    FindLayout L;
    memset(&L, 0, sizeof(L));
    FindWs& c = L.caps;
    const int64_t nmid = mn(N, S / (kSmallMaxMin + 1));
    const int64_t nsb = mn(N, S / (kSortWaveMax + 1));
    const int64_t nbig = mn(N, S / (kMidMax + 1));
    c.cap_small = N + 1;
    c.cap_dmid = nmid + 1;
    c.cap_imid = mn(P, K * nmid) + 1;
    c.cap_dsb = nsb + 1;
    c.cap_isb = mn(P, K * nsb) + 1;
    c.cap_dbig = nbig + 1;
    // the XCD-local layout pads a node's items to whole quads of projections
    // times whole groups of kXcds chunks, plus alignment
    c.cap_ibiga = (K + 3) * (S / kChunk + 2 * kXcds * nbig) + 4 * kXcds * nbig + 1;
    c.cap_ibigc = mn(P, K * nbig) + 1;
    c.cap_slots = mn(P, K * nsb) + 1;
    c.cap_bigslots = mn(P, K * nbig) + 1;
    const int64_t nmid2 = mn(N, S / (kMidSplitMin + 1));
    c.cap_dmid2 = nmid2 + 1;
    c.cap_imid2 = mn(P, K * nmid2) + 1;
    // every big node's n * k values, each node rounded up to whole units; off
    // (0) beyond 2^30 units (a terabyte), where nodes fall back to re-gathering
    c.cap_vcache = nbig > 0 ? (S * K) / kVcUnit + nbig + 1 : 0;
    if (c.cap_vcache > (int64_t(1) << 30) || !vcache) c.cap_vcache = 0;
    c.cap_flnk = flnk_entries;
    size_t o = 0;
    L.hdr = o; o = align_up(o + H_COUNT * sizeof(int32_t));
    L.small_items = o; o = align_up(o + c.cap_small * sizeof(int4));
    L.desc_mid = o; o = align_up(o + c.cap_dmid * sizeof(int4));
    L.desc_mid2 = o; o = align_up(o + c.cap_dmid2 * sizeof(int4));
    L.desc_sb = o; o = align_up(o + c.cap_dsb * sizeof(int4));
    L.desc_big = o; o = align_up(o + 2 * c.cap_dbig * sizeof(int4));
    L.items_mid = o; o = align_up(o + c.cap_imid * 2 * sizeof(int4));
    L.items_mid2 = o; o = align_up(o + c.cap_imid2 * 2 * sizeof(int4));
    L.items_sb = o; o = align_up(o + c.cap_isb * sizeof(int2));
    L.items_biga = o; o = align_up(o + c.cap_ibiga * sizeof(int2));
    L.items_bigc = o; o = align_up(o + c.cap_ibigc * sizeof(int2));
    L.slots = o; o = align_up(o + c.cap_slots * 80);
    L.crange = o; o = align_up(o + c.cap_ibiga * sizeof(float2));
    L.brange = o; o = align_up(o + c.cap_bigslots * sizeof(float2));
    L.phist = o; o = align_up(o + (size_t)c.cap_bigslots * bins * classes * sizeof(int32_t));
    L.vcache = o; o = align_up(o + (size_t)c.cap_vcache * kVcUnit * sizeof(float));
    L.flnk = o; o = align_up(o + (size_t)c.cap_flnk * sizeof(double));
    L.total = o;
    return L;
}

void sof::find_bind(const FindLayout& L, void* ws, FindWs* w) {
    char* b = (char*)ws;
    *w = L.caps;
    w->hdr = (int32_t*)(b + L.hdr);
    w->small_items = (int4*)(b + L.small_items);
    w->desc_mid = (int4*)(b + L.desc_mid);
    w->desc_mid2 = (int4*)(b + L.desc_mid2);
    w->desc_sb = (int4*)(b + L.desc_sb);
    w->desc_big = (int4*)(b + L.desc_big);
    w->items_mid = (int4*)(b + L.items_mid);
    w->items_mid2 = (int4*)(b + L.items_mid2);
    w->items_sb = (int2*)(b + L.items_sb);
    w->items_biga = (int2*)(b + L.items_biga);
    w->items_bigc = (int2*)(b + L.items_bigc);
    w->slots = (void*)(b + L.slots);
    w->crange = (float2*)(b + L.crange);
    w->brange = (float2*)(b + L.brange);
    w->phist = (int32_t*)(b + L.phist);
    w->vcache = (float*)(b + L.vcache);
    w->flnk = (double*)(b + L.flnk);
}

extern "C" int sof_workspace_size(const sof_ctx* ctx, const sof_data* data, const sof_frontier* fr,
                                  const sof_proj* proj, const sof_params* params, size_t* bytes) {
    (void)ctx;
    if (!bytes) return fail(SOF_ERR_INVALID_ARG, "bytes is NULL");
    int rc;
    if ((rc = check_data(data)) || (rc = check_frontier(fr)) || (rc = check_proj(proj, data)) ||
        (rc = check_params(params)))
        return rc;
    FindLayout L = find_layout(fr->n_nodes, fr->n_samples, proj->n_proj, proj->max_proj_per_node,
                               params->bins, data->n_classes,
                               flnk_entries(params->criterion, fr->max_node_samples));
    size_t need = L.total;
    size_t part = part_workspace(fr->n_nodes, fr->n_samples);
    if (part > need) need = part;
    size_t pj = project_workspace(fr->n_nodes, fr->n_samples, proj->n_proj);
    if (pj > need) need = pj;
    *bytes = need;
    return SOF_OK;
}

static int check_ws(void* ws, size_t ws_bytes, size_t need) {
    if (need == 0) return SOF_OK;
    if (!ws) return fail(SOF_ERR_WORKSPACE, "workspace is NULL (need %zu bytes)", need);
    if (((uintptr_t)ws) % SOF_WORKSPACE_ALIGN)
        return fail(SOF_ERR_WORKSPACE, "workspace not %d-byte aligned", SOF_WORKSPACE_ALIGN);
    if (ws_bytes < need)
        return fail(SOF_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    return SOF_OK;
}

int sof::check_ws_public(void* ws, size_t ws_bytes, size_t need) { return check_ws(ws, ws_bytes, need); }

// ---------------------------------------------------------------------------
// find splits

int sof::fill_find_args(const sof_data* data, const sof_frontier* fr, const sof_params* params,
                        sof_split* out, int32_t* hist_out, FindArgs* a) {
    memset(a, 0, sizeof(*a));
    a->x = data->x;
    a->ld = data->ld;
    a->y = data->y;
    a->n_rows = data->n_rows;
    a->n_features = data->n_features;
    a->n_classes = data->n_classes;
    a->dtype = data->dtype;
    a->node_offsets = fr->node_offsets;
    a->sample_idx = fr->sample_idx;
    a->n_samples = fr->n_samples;
    a->n_nodes = fr->n_nodes;
    a->n_nodes_dev = nullptr;
    a->node_bins = params->node_bins;
    a->bins = params->bins;
    a->sort_threshold = clamp_threshold(params->sort_threshold);
    a->small_max = params->small_max ? params->small_max : kSmallMax;
    a->mid_split = params->mid_split ? params->mid_split : kMidSplit;
    a->bin_mode = params->bin_mode;
    a->criterion = params->criterion;
    a->bin_seed = params->bin_seed;
    a->out = out;
    a->hist_out = hist_out;
    return SOF_OK;
}

extern "C" int sof_find_splits(sof_ctx* ctx, const sof_data* data, const sof_frontier* fr,
                               const sof_proj* proj, const sof_params* params, sof_split* out,
                               int32_t* hist_out, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx) return fail(SOF_ERR_INVALID_ARG, "ctx is NULL");
    int rc;
    if ((rc = check_data(data)) || (rc = check_frontier(fr)) || (rc = check_proj(proj, data)) ||
        (rc = check_params(params)))
        return rc;
    if (fr->n_nodes > 0 && !out) return fail(SOF_ERR_INVALID_ARG, "out is NULL");
    FindLayout L = find_layout(fr->n_nodes, fr->n_samples, proj->n_proj, proj->max_proj_per_node,
                               params->bins, data->n_classes,
                               flnk_entries(params->criterion, fr->max_node_samples));
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    if (fr->n_nodes == 0) return SOF_OK;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    LaunchCfg cfg;
    if ((rc = launch_cfg(ctx, params->bins, data->n_classes,
                         (params->bin_mode == SOF_BINS_RANDOM ? 1 : 0) | (params->criterion == SOF_CRIT_ENTROPY ? 2 : 0),
                         &cfg)))
        return rc;
    if (ctx->check && (rc = device_check(ctx, data, fr, proj, params, (hipStream_t)stream))) return rc;
    FindArgs a;
    fill_find_args(data, fr, params, out, hist_out, &a);
    find_bind(L, ws, &a.ws);
    ProjCSR p{proj->proj_offsets, proj->nz_offsets, proj->nz_feature, proj->nz_weight, proj->n_proj,
              proj->n_nz, proj->nz_value};
    {
        std::lock_guard<std::mutex> g(ctx->launch_mu);
        e = launch_find_csr(a, p, cfg, find_streams(ctx, (hipStream_t)stream), timing_events(ctx));
    }
    if (e != hipSuccess) return hip_fail(e, "find_splits launch");
    return SOF_OK;
}

// The same launch sequence as sof_find_splits, with the workspace in the
// device's static scratch array instead of a caller buffer: no allocation,
// no projected-value cache (big nodes re-gather their columns), and no
// SOF_CHECK content checks (they allocate a flag).  The sequence clears the
// queue counters itself and overwrites everything else it reads, so stale
// contents of an earlier call do no harm; calls that overlap on one device
// share the array and race.
extern "C" int sof_find_splits_noalloc(sof_ctx* ctx, const sof_data* data, const sof_frontier* fr,
                                       const sof_proj* proj, const sof_params* params, sof_split* out,
                                       int32_t* hist_out, void* stream) {
    if (!ctx) return fail(SOF_ERR_INVALID_ARG, "ctx is NULL");
    int rc;
    if ((rc = check_data(data)) || (rc = check_frontier(fr)) || (rc = check_proj(proj, data)) ||
        (rc = check_params(params)))
        return rc;
    if (fr->n_nodes > 0 && !out) return fail(SOF_ERR_INVALID_ARG, "out is NULL");
    FindLayout L = find_layout(fr->n_nodes, fr->n_samples, proj->n_proj, proj->max_proj_per_node,
                               params->bins, data->n_classes,
                               flnk_entries(params->criterion, fr->max_node_samples), false);
    if (L.total > (size_t)SOF_STATIC_SCRATCH_BYTES)
        return fail(SOF_ERR_WORKSPACE,
                    "sof_find_splits_noalloc: these sizes need %zu bytes of scratch, above the static %zu",
                    L.total, (size_t)SOF_STATIC_SCRATCH_BYTES);
    if (!ctx->scratch) return fail(SOF_ERR_HIP, "sof_find_splits_noalloc: no static scratch on this device");
    if (fr->n_nodes == 0) return SOF_OK;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    LaunchCfg cfg;
    if ((rc = launch_cfg(ctx, params->bins, data->n_classes,
                         (params->bin_mode == SOF_BINS_RANDOM ? 1 : 0) | (params->criterion == SOF_CRIT_ENTROPY ? 2 : 0),
                         &cfg)))
        return rc;
    FindArgs a;
    fill_find_args(data, fr, params, out, hist_out, &a);
    find_bind(L, ctx->scratch, &a.ws);
    ProjCSR p{proj->proj_offsets, proj->nz_offsets, proj->nz_feature, proj->nz_weight, proj->n_proj,
              proj->n_nz, proj->nz_value};
    {
        std::lock_guard<std::mutex> g(ctx->launch_mu);
        e = launch_find_csr(a, p, cfg, find_streams(ctx, (hipStream_t)stream), nullptr);
    }
    if (e != hipSuccess) return hip_fail(e, "find_splits launch");
    return SOF_OK;
}
