// k_partition.hip -- stable partition of every node's samples by its split
// (paper section 4: each node splits its samples between its children).
//
// The split rule is re-evaluated on recomputed projected values (the same FP32
// CSR-order sums as the search): equal-width histogram splits send v left iff
// bin(v) <= bin, random-width ones iff v < threshold (the next boundary, which
// is the same rule), sort splits iff v <= threshold.  Output per node: left
// samples in input order, then right samples in input order.
//
//   k_pplan     per node: child offsets, tiny/small-node queues or chunk items
//   k_ptiny     nodes <= 1024 samples: one wave per node, all in registers
//   k_psmall    nodes <= 2048 samples: one block per node, 8 samples per
//               thread, scattered from registers
//   k_ppred     chunk items (2048 samples) of larger nodes: predicate bits
//               and left counts (first pass)
//   k_pchunkscan  one block: exclusive prefix of the chunk items' left counts
//   k_pscatter  chunk items: left counts of the node's earlier chunks from
//               that prefix, scatter
// The three node classes are independent: after the plan, k_ptiny and the
// chunk chain (k_ppred, k_pchunkscan, k_pscatter) run on the context's two
// auxiliary streams beside k_psmall on the caller's, and join it at the end.
// Every gather requests all (up to 4) columns of the split's projection in
// one round trip.
#include <cstring>

#include "sof_device.h"
#include "sof_host.h"
#include "sof_internal.h"
#include "sof_sampler.h"

namespace sof {


constexpr int kPartTiny = 1024;            // one wave per node up to here
constexpr int kPartMax = 2048;             // one block per node up to here; chunk size above
constexpr int kPR = kPartMax / kBlock;     // 8 samples per thread
constexpr int kWordsPerChunk = kPartMax / kWave;

enum { P_SMALL = 0, P_ITEMS, P_TINY, P_Q_SMALL = 8, P_Q_A, P_Q_B, P_Q_TINY, P_COUNT = 16 };

__device__ __forceinline__ void wave_sync_p() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int64_t clampp(int64_t x, int64_t lo, int64_t hi) {
    return x < lo ? lo : (x > hi ? hi : x);
}

__device__ __forceinline__ int nodes_of(const PartArgs& A) {
    if (!A.n_nodes_dev) return A.n_nodes;
    int n = *A.n_nodes_dev;
    return n < 0 ? 0 : (n > A.n_nodes ? A.n_nodes : n);
}

__device__ __forceinline__ void prange(const PartArgs& A, int v, int64_t& s0, int64_t& n) {
    int64_t a = clampp(A.node_offsets[v], 0, A.n_samples);
    int64_t b = clampp(A.node_offsets[v + 1], a, A.n_samples);
    s0 = a;
    n = b - a;
}


// projection sources (same contracts as in the search)
__device__ __forceinline__ int pcount(const ProjCSR& P, int v) {
    int a = (int)clampp(P.proj_offsets[v], 0, P.n_proj);
    int b = (int)clampp(P.proj_offsets[v + 1], a, P.n_proj);
    return b - a;
}
__device__ __forceinline__ int pstage(const ProjCSR& P, int v, int p, int d, int32_t* lf, uint32_t* ls) {
    int q = (int)clampp(P.proj_offsets[v], 0, P.n_proj) + p;
    int64_t j0 = clampp(P.nz_offsets[q], 0, P.n_nz);
    int64_t j1 = clampp(P.nz_offsets[q + 1], j0, P.n_nz);
    if (j1 - j0 > SOF_MAX_NNZ) j1 = j0 + SOF_MAX_NNZ;
    int z = (int)(j1 - j0);
    int lane = lane_id();
    if (lane < z) {
        uint32_t f = (uint32_t)P.nz_feature[j0 + lane];
        lf[lane] = f < (uint32_t)d ? (int)f : 0;
        ls[lane] = csr_weight_bits(P, j0 + lane);
    }
    wave_sync_p();
    return z;
}

__device__ __forceinline__ int pcount(const ProjHash& P, int) { return P.k; }
__device__ __forceinline__ int pstage(const ProjHash& P, int v, int p, int d, int32_t* lf, uint32_t* ls) {
    const int lane = lane_id();
    const SampSpec sp{P.seed, d, P.z, P.mode, P.wmode};
    const int tree = P.tree_of[v], pos = P.pos_of[v], level = *P.level;
    const int z = __builtin_amdgcn_readfirstlane(samp_nnz(sp, tree, level, pos, p));
    int mine, rank;
    samp_wave(sp, z, tree, level, pos, p, mine, rank);
    if (lane < z) {
        lf[rank] = mine;
        ls[rank] = samp_weight_bits(sp, tree, level, pos, p, rank);
    }
    wave_sync_p();
    return z;
}

// The split projection in registers: lane j < z holds the j-th feature
// (ascending order) and its sign bit; returns z.
__device__ __forceinline__ int preg(const ProjCSR& P, int v, int p, int d, int& fj, uint32_t& sj) {
    int q = (int)clampp(P.proj_offsets[v], 0, P.n_proj) + p;
    int64_t j0 = clampp(P.nz_offsets[q], 0, P.n_nz);
    int64_t j1 = clampp(P.nz_offsets[q + 1], j0, P.n_nz);
    if (j1 - j0 > SOF_MAX_NNZ) j1 = j0 + SOF_MAX_NNZ;
    const int z = (int)(j1 - j0);
    const int lane = lane_id();
    fj = 0;
    sj = 0;
    if (lane < z) {
        uint32_t f = (uint32_t)P.nz_feature[j0 + lane];
        fj = f < (uint32_t)d ? (int)f : 0;
        sj = csr_weight_bits(P, j0 + lane);
    }
    return z;
}
__device__ __forceinline__ int preg(const ProjHash& P, int v, int p, int d, int& fj, uint32_t& sj) {
    const int lane = lane_id();
    const SampSpec sp{P.seed, d, P.z, P.mode, P.wmode};
    const int tree = P.tree_of[v], pos = P.pos_of[v], level = *P.level;
    const int z = __builtin_amdgcn_readfirstlane(samp_nnz(sp, tree, level, pos, p));
    int mine, rank;
    samp_wave(sp, z, tree, level, pos, p, mine, rank);
    // lane j takes the draw of rank j
    fj = 0;
    for (int i = 0; i < z; ++i) {
        const int ri = __shfl(rank, i), mi = __shfl(mine, i);
        if (ri == lane) fj = mi;
    }
    sj = lane < z ? samp_weight_bits(sp, tree, level, pos, p, lane) : 0u;
    return z;
}

// One wave partitions a node of n <= 64 R samples: each lane holds R samples
// (sample i at lane i mod 64, row i / 64), the left masks of the R rows stay
// in scalar registers, and each sample goes straight to its destination.
// Slots past the end repeat the last sample so every column load is issued at
// a valid address.
template <typename T, class PS, int R>
__device__ void ptiny_r(const PartArgs& A, const PS& P, int v, int64_t s0, int n) {
    const int lane = lane_id();
    const SplitRec sp = ((const SplitRec*)A.splits)[v];
    const int k = pcount(P, v);
    const bool all_left = sp.proj < 0 || sp.proj >= k;
    int fj = 0;
    uint32_t sj = 0;
    const int z = __builtin_amdgcn_readfirstlane(all_left ? 0 : preg(P, v, sp.proj, A.n_features, fj, sj));
    int B = A.bins;
    if (A.node_bins) {
        int b = A.node_bins[v];
        B = b < 2 ? 2 : (b > A.bins ? A.bins : b);
    }
    int32_t raw[R];
    uint32_t off[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = lane + r * kWave;
        raw[r] = A.sample_idx[s0 + (i < n ? i : n - 1)];
        const uint32_t row = (uint32_t)raw[r] < (uint32_t)A.n_rows ? (uint32_t)raw[r] : 0u;
        off[r] = row * (uint32_t)sizeof(T);
    }
    // FB columns per round trip (a round's spare slots re-read its first
    // column, a valid address, and are not added); adds in CSR order
    constexpr int FB = R <= 8 ? 4 : 2;
    float val[R];
#pragma unroll
    for (int r = 0; r < R; ++r) val[r] = 0.f;
    for (int j = 0; j < z; j += FB) {
        const int nf = z - j < FB ? z - j : FB;
        float x[FB][R];
        uint32_t sg[FB];
#pragma unroll
        for (int t = 0; t < FB; ++t) {
            const int jt = t < nf ? j + t : j;
            const int f = __builtin_amdgcn_readlane(fj, jt);
            sg[t] = (uint32_t)__builtin_amdgcn_readlane((int)sj, jt);
            const T* col = (const T*)A.x + (int64_t)f * A.ld;
#pragma unroll
            for (int r = 0; r < R; ++r) x[t][r] = ldx((const T*)((const char*)col + off[r]), 0);
        }
#pragma unroll
        for (int t = 0; t < FB; ++t) {
            if (t >= nf) break;
#pragma unroll
            for (int r = 0; r < R; ++r) val[r] = __fadd_rn(val[r], weighted_term(x[t][r], sg[t]));
        }
    }
    uint64_t m[R];
    int nl = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = lane + r * kWave;
        bool left = true;
        if (!all_left)
            left = sp.kind == SOF_SPLIT_HIST    ? bin_index(val[r], sp.lo, sp.scale, B) <= sp.bin
                   : sp.kind == SOF_SPLIT_RHIST ? val[r] < sp.threshold
                                                : val[r] <= sp.threshold;
        m[r] = __ballot(i < n && left);
        nl += __popcll(m[r]);
    }
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    int lpre = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = lane + r * kWave;
        const int64_t dst = ((m[r] >> lane) & 1ull) ? s0 + lpre + __popcll(m[r] & below)
                                                    : s0 + nl + (r * kWave - lpre) + __popcll(~m[r] & below);
        if (i < n && dst >= s0 && dst < s0 + n) A.out_idx[dst] = raw[r];
        lpre += __popcll(m[r]);
    }
    A.child_offsets[2 * v + 1] = (int32_t)(s0 + nl);   // every lane stores the same value
}

// Tiny nodes are dealt to waves round-robin (no queue): every value that
// steers the loop is read into a scalar register, and no lane-subset branch
// precedes a cross-lane operation, so the wave stays converged throughout.
template <typename T, class PS>
__global__ __launch_bounds__(kBlock) void k_ptiny(PartArgs A, PS P) {
    const int ntiny = __builtin_amdgcn_readfirstlane(A.hdr[P_TINY]);
    const int N = nodes_of(A);
    const int wave = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6)));
    const int nwaves = (int)gridDim.x * kWavesPerBlock;
    for (int it = wave; it < ntiny; it += nwaves) {
        const int v = __builtin_amdgcn_readfirstlane(A.big_items[A.cap_items + A.n_nodes - 1 - it].x);
        if (v < 0 || v >= N) continue;
        int64_t s0, n;
        prange(A, v, s0, n);
        const int s0u = __builtin_amdgcn_readfirstlane((int)s0);
        const int nu = __builtin_amdgcn_readfirstlane((int)n);
        if (nu <= 0) A.child_offsets[2 * v + 1] = s0u;   // every lane stores the same value
        else if (nu <= 64) ptiny_r<T, PS, 1>(A, P, v, s0u, nu);
        else if (nu <= 128) ptiny_r<T, PS, 2>(A, P, v, s0u, nu);
        else if (nu <= 256) ptiny_r<T, PS, 4>(A, P, v, s0u, nu);
        else if (nu <= 512) ptiny_r<T, PS, 8>(A, P, v, s0u, nu);
        else ptiny_r<T, PS, 16>(A, P, v, s0u, nu < kPartTiny ? nu : kPartTiny);
    }
}

struct PShared {
    int item;
    int z;
    int nleft;
    int pad;
    int64_t base[2];
    int32_t lf[16];
    uint32_t ls[16];
    int32_t cnt[kPR][kWavesPerBlock];
    int32_t pre[kPR][kWavesPerBlock];
    uint64_t mask[kPR][kWavesPerBlock];
};

// Predicate bits of up to 8192 samples starting at sample position `at`
// (row r of 256 samples, wave w: bit lane of mask[r][w]), with R >= the
// number of 256-sample rows.  Slots past the end repeat the last sample, so
// the loads of one column are issued together at valid addresses; their
// predicate bits are cleared by the i < cn test.
template <typename T, class PS, int R>
__device__ void predicates_r(const PartArgs& A, const PS& P, int v, int64_t at, int64_t cn, PShared& S,
                             uint32_t (&rid)[R]) {
    const int tid = threadIdx.x, w = tid >> 6;
    const SplitRec sp = ((const SplitRec*)A.splits)[v];
    const int k = pcount(P, v);
    const bool all_left = sp.proj < 0 || sp.proj >= k;
    // the row ids (rid: as stored in sample_idx) are requested before the
    // split's projection is staged
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = tid + (int64_t)r * kBlock;
        rid[r] = cn > 0 ? (uint32_t)A.sample_idx[at + (i < cn ? i : cn - 1)] : 0u;
    }
    if (w == 0) {
        int z = all_left ? 0 : pstage(P, v, sp.proj, A.n_features, S.lf, S.ls);
        if (lane_id() == 0) S.z = z;
    }
    __syncthreads();
    const int z = __builtin_amdgcn_readfirstlane(S.z);
    int B = A.bins;
    if (A.node_bins) {
        int b = A.node_bins[v];
        B = b < 2 ? 2 : (b > A.bins ? A.bins : b);
    }
    uint32_t off[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = rid[r] < (uint32_t)A.n_rows ? (int)rid[r] : 0;
        off[r] = (uint32_t)row * (uint32_t)sizeof(T);
    }
    // FB columns per round trip (all loads of a round at valid addresses; a
    // round's spare slots re-read its first column and are not added); the
    // adds stay in CSR order
    constexpr int FB = R <= 8 ? 4 : (R <= 16 ? 2 : 1);
    float val[R];
#pragma unroll
    for (int r = 0; r < R; ++r) val[r] = 0.f;
    for (int j = 0; j < z; j += FB) {
        const int nf = z - j < FB ? z - j : FB;
        float x[FB][R];
        uint32_t sg[FB];
#pragma unroll
        for (int t = 0; t < FB; ++t) {
            const int jt = t < nf ? j + t : j;
            const int f = __builtin_amdgcn_readfirstlane(S.lf[jt]);
            sg[t] = __builtin_amdgcn_readfirstlane(S.ls[jt]);
            const T* col = (const T*)A.x + (int64_t)f * A.ld;
#pragma unroll
            for (int r = 0; r < R; ++r) x[t][r] = ldx((const T*)((const char*)col + off[r]), 0);
        }
#pragma unroll
        for (int t = 0; t < FB; ++t) {
            if (t >= nf) break;
#pragma unroll
            for (int r = 0; r < R; ++r) val[r] = __fadd_rn(val[r], weighted_term(x[t][r], sg[t]));
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = tid + (int64_t)r * kBlock;
        bool left = true;
        if (!all_left)
            left = sp.kind == SOF_SPLIT_HIST    ? bin_index(val[r], sp.lo, sp.scale, B) <= sp.bin
                   : sp.kind == SOF_SPLIT_RHIST ? val[r] < sp.threshold
                                                : val[r] <= sp.threshold;
        const uint64_t m = __ballot(i < cn && left);
        if (lane_id() == 0) {
            S.mask[r][w] = m;
            S.cnt[r][w] = __popcll(m);
        }
    }
    __syncthreads();
}

template <typename T, class PS, int R>
__device__ void predicates_chunk_r(const PartArgs& A, const PS& P, int v, int64_t at, int64_t cn, PShared& S) {
    uint32_t rid[R];
    predicates_r<T, PS, R>(A, P, v, at, cn, S, rid);
}
template <typename T, class PS>
__device__ void predicates(const PartArgs& A, const PS& P, int v, int64_t at, int64_t cn, PShared& S) {
    const int nr = (int)((cn + kBlock - 1) / kBlock);
    if (nr <= 1) predicates_chunk_r<T, PS, 1>(A, P, v, at, cn, S);
    else if (nr <= 2) predicates_chunk_r<T, PS, 2>(A, P, v, at, cn, S);
    else if (nr <= 4) predicates_chunk_r<T, PS, 4>(A, P, v, at, cn, S);
    else predicates_chunk_r<T, PS, kPR>(A, P, v, at, cn, S);
}

// Exclusive prefix of S.cnt in (row, wave) order; returns the total.
__device__ int row_prefix(PShared& S, int nr) {
    const int tid = threadIdx.x;
    if (tid < kWave) {
        // lane l owns entries 2l, 2l+1 of the row-major (row, wave) list
        int e0 = 2 * tid, e1 = 2 * tid + 1;
        int c0 = e0 < nr * kWavesPerBlock ? S.cnt[e0 >> 2][e0 & 3] : 0;
        int c1 = e1 < nr * kWavesPerBlock ? S.cnt[e1 >> 2][e1 & 3] : 0;
        uint32_t incl = wave_incl_scan((uint32_t)(c0 + c1));
        uint32_t ex = incl - (uint32_t)(c0 + c1);
        if (e0 < kPR * kWavesPerBlock) S.pre[e0 >> 2][e0 & 3] = (int)ex;
        if (e1 < kPR * kWavesPerBlock) S.pre[e1 >> 2][e1 & 3] = (int)ex + c0;
        if (tid == 63) S.nleft = (int)incl;
    }
    __syncthreads();
    return S.nleft;
}

// Scatter the chunk's samples given the left block base and right block base;
// destinations outside the node's range [lo, hi) (possible only for
// inconsistent offsets) are dropped.
__device__ void scatter(const PartArgs& A, PShared& S, int64_t at, int64_t cn, int64_t lbase,
                        int64_t rbase, int64_t lo, int64_t hi) {
    const int tid = threadIdx.x, w = tid >> 6, lane = lane_id();
    const int nr = (int)((cn + kBlock - 1) / kBlock);
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < nr; ++r) {
        int64_t i = tid + (int64_t)r * kBlock;
        if (i >= cn) continue;
        const uint64_t m = S.mask[r][w];
        const int lpre = S.pre[r][w];
        const int64_t before = (int64_t)r * kBlock + w * kWave;   // samples before this wave's first
        const int32_t row = A.sample_idx[at + i];
        const int64_t dst = ((m >> lane) & 1ull) ? lbase + lpre + __popcll(m & below)
                                                 : rbase + (before - lpre) + __popcll(~m & below);
        if (dst >= lo && dst < hi) A.out_idx[dst] = row;
    }
}

// A whole node of n <= kPartMax samples by one block: predicate bits, the
// block's prefix of left counts, then every sample goes from its register
// straight to its destination.
template <typename T, class PS, int R>
__device__ void psmall_node_r(const PartArgs& A, const PS& P, int v, int64_t s0, int64_t n, PShared& S) {
    uint32_t rid[R];
    predicates_r<T, PS, R>(A, P, v, s0, n, S, rid);
    const int nr = (int)((n + kBlock - 1) / kBlock);
    const int nl = row_prefix(S, nr);
    const int tid = threadIdx.x, w = tid >> 6, lane = lane_id();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = tid + (int64_t)r * kBlock;
        if (i >= n) continue;
        const uint64_t m = S.mask[r][w];
        const int lpre = S.pre[r][w];
        const int64_t before = (int64_t)r * kBlock + w * kWave;   // samples before this wave's first
        const int64_t dst = ((m >> lane) & 1ull) ? s0 + lpre + __popcll(m & below)
                                                 : s0 + nl + (before - lpre) + __popcll(~m & below);
        if (dst >= s0 && dst < s0 + n) A.out_idx[dst] = (int32_t)rid[r];
    }
    if (tid == 0) A.child_offsets[2 * v + 1] = (int32_t)(s0 + nl);
}
template <typename T, class PS>
__device__ void psmall_node(const PartArgs& A, const PS& P, int v, int64_t s0, int64_t n, PShared& S) {
    const int nr = (int)((n + kBlock - 1) / kBlock);
    if (nr <= 4) psmall_node_r<T, PS, 4>(A, P, v, s0, n, S);
    else psmall_node_r<T, PS, kPR>(A, P, v, s0, n, S);
}

template <class PS>
__global__ __launch_bounds__(kBlock) void k_pplan(PartArgs A, PS P) {
    const int N = nodes_of(A);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        A.child_offsets[2 * N] = (int32_t)clampp(A.node_offsets[N], 0, A.n_samples);
    // the grid covers the nodes in whole waves, so every lane reaches the
    // wave-wide allocation
    for (int v0 = blockIdx.x * kBlock; v0 < N; v0 += gridDim.x * kBlock) {
        const int v = v0 + threadIdx.x;
        const bool act = v < N;
        int64_t s0 = 0, n = 0;
        if (act) {
            prange(A, v, s0, n);
            A.child_offsets[2 * v] = (int32_t)s0;
        }
        const int nch = act && n > kPartMax ? (int)((n + kPartMax - 1) / kPartMax) : 0;
        const int ctr[3] = {P_TINY, P_SMALL, P_ITEMS};
        const int cnt[3] = {act && n <= kPartTiny, act && n > kPartTiny && n <= kPartMax, nch};
        int o[3];
        wave_alloc_n<3>(A.hdr, ctr, cnt, o);
        // the chunk items of the wave's large nodes, written by the whole wave
        const int lane = lane_id();
        uint64_t big = __ballot(nch > 0);
        while (big) {
            const int src = __builtin_ctzll(big);
            big &= big - 1;
            const int bv = __builtin_amdgcn_readlane(v, src);
            const int bn = __builtin_amdgcn_readlane(nch, src);
            const int bb = __builtin_amdgcn_readlane(o[2], src);
            for (int c = lane; c < bn; c += kWave)
                if (bb + (int64_t)c < A.cap_items) A.big_items[bb + c] = make_int4(bv, c, bn, bb);
        }
        if (!act) continue;
        if (n <= kPartTiny) {
            // tiny list fills the node-list region from its far end
            A.big_items[A.cap_items + A.n_nodes - 1 - o[0]] = make_int4(v, 0, 0, 0);
        } else if (n <= kPartMax) {
            A.big_items[A.cap_items + o[1]] = make_int4(v, 0, 0, 0);   // small list lives after the items
        }
    }
}

template <typename T, class PS>
__global__ __launch_bounds__(kBlock) void k_psmall(PartArgs A, PS P) {
    extern __shared__ __align__(16) char smem[];
    PShared& S = *(PShared*)smem;
    const int nsmall = A.hdr[P_SMALL];
    const int N = nodes_of(A);
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) S.item = atomicAdd(&A.hdr[P_Q_SMALL], 1);
        __syncthreads();
        const int it = S.item;
        if (it >= nsmall) break;
        const int v = A.big_items[A.cap_items + it].x;
        if (v < 0 || v >= N) continue;
        int64_t s0, n;
        prange(A, v, s0, n);
        if (n > kPartMax) n = kPartMax;   // the plan never queues larger nodes here
        psmall_node<T>(A, P, v, s0, n, S);
    }
}

template <typename T, class PS>
__global__ __launch_bounds__(kBlock) void k_ppred(PartArgs A, PS P) {
    extern __shared__ __align__(16) char smem[];
    PShared& S = *(PShared*)smem;
    const int nitems = (int)min((int64_t)A.hdr[P_ITEMS], A.cap_items);
    const int N = nodes_of(A);
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) S.item = atomicAdd(&A.hdr[P_Q_A], 1);
        __syncthreads();
        const int e = S.item;
        if (e >= nitems) break;
        const int4 d = A.big_items[e];
        if (d.x < 0 || d.x >= N) continue;
        int64_t s0, n;
        prange(A, d.x, s0, n);
        const int64_t c0 = (int64_t)d.y * kPartMax;
        int64_t cn = n - c0;
        cn = cn < 0 ? 0 : (cn > kPartMax ? kPartMax : cn);
        predicates<T>(A, P, d.x, s0 + c0, cn, S);
        const int tid = threadIdx.x;
        if (tid < kWordsPerChunk) {
            A.pred_bits[(int64_t)e * kWordsPerChunk + tid] = S.mask[tid >> 2][tid & 3];
        }
        if (tid == 0) {
            int s = 0;
            const int nr = (int)((cn + kBlock - 1) / kBlock);
            for (int r = 0; r < nr; ++r)
                for (int w = 0; w < kWavesPerBlock; ++w) s += S.cnt[r][w];
            A.chunk_left[e] = s;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_pscatter(PartArgs A) {
    extern __shared__ __align__(16) char smem[];
    PShared& S = *(PShared*)smem;
    int64_t* s_base = S.base;
    const int nitems = (int)min((int64_t)A.hdr[P_ITEMS], A.cap_items);
    const int N = nodes_of(A);
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) S.item = atomicAdd(&A.hdr[P_Q_B], 1);
        __syncthreads();
        const int e = S.item;
        if (e >= nitems) break;
        const int4 d = A.big_items[e];
        if (d.x < 0 || d.x >= N) continue;
        int64_t s0, n;
        prange(A, d.x, s0, n);
        const int64_t c0 = (int64_t)d.y * kPartMax;
        int64_t cn = n - c0;
        cn = cn < 0 ? 0 : (cn > kPartMax ? kPartMax : cn);
        const int tid = threadIdx.x;
        // left counts of the node's chunks before this one, and in total, from
        // the exclusive prefix over all chunk items (a node's items are
        // consecutive, from d.w)
        if (tid == 0) {
            const int64_t first = clampp(d.w, 0, nitems);
            const int64_t last = clampp((int64_t)d.w + d.z, first, nitems);
            const int64_t pf = A.chunk_pre[first];
            s_base[0] = A.chunk_pre[clampp(e, first, last)] - pf;
            s_base[1] = A.chunk_pre[last] - pf;
        }
        if (tid < kWordsPerChunk) {
            uint64_t m = A.pred_bits[(int64_t)e * kWordsPerChunk + tid];
            S.mask[tid >> 2][tid & 3] = m;
            S.cnt[tid >> 2][tid & 3] = __popcll(m);
        }
        __syncthreads();
        const int nr = (int)((cn + kBlock - 1) / kBlock);
        row_prefix(S, nr);
        const int64_t before = s_base[0], total = s_base[1];
        scatter(A, S, s0 + c0, cn, s0 + before, s0 + total + (c0 - before), s0, s0 + n);
        if (tid == 0 && d.y == 0) A.child_offsets[2 * d.x + 1] = (int32_t)(s0 + total);
    }
}

// Exclusive prefix of the chunk items' left counts (pre[0 .. nitems], 64-bit),
// by one block: tiles of kBlock * 4 items, each thread summing 4 consecutive
// counts, a block scan of the thread sums, and a carry across tiles.
__global__ __launch_bounds__(kBlock) void k_pchunkscan(PartArgs A) {
    __shared__ int64_t wsum[kWavesPerBlock];
    const int nitems = (int)min((int64_t)A.hdr[P_ITEMS], A.cap_items);
    const int tid = threadIdx.x, w = tid >> 6, lane = lane_id();
    int64_t carry = 0;
    for (int t0 = 0; t0 < nitems; t0 += kBlock * 4) {
        int64_t c[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = t0 + tid * 4 + i;
            c[i] = e < nitems ? (int64_t)A.chunk_left[e] : 0;
        }
        const int64_t mine = c[0] + c[1] + c[2] + c[3];
        int64_t x = mine;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int64_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == kWave - 1) wsum[w] = x;
        __syncthreads();
        int64_t before = carry, tile = 0;
        for (int j = 0; j < kWavesPerBlock; ++j) {
            if (j < w) before += wsum[j];
            tile += wsum[j];
        }
        int64_t run = before + x - mine;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = t0 + tid * 4 + i;
            if (e < nitems) A.chunk_pre[e] = run;
            run += c[i];
        }
        carry += tile;
        __syncthreads();
    }
    if (tid == 0) A.chunk_pre[nitems] = carry;
}

__global__ void k_preset(int32_t* hdr) {
    for (int i = threadIdx.x; i < P_COUNT; i += blockDim.x) hdr[i] = 0;
}

template <typename T, class PS>
hipError_t launch_part_t(const PartArgs& a, const PS& p, int n_cu, const FindStreams& st) {
    const hipStream_t s = st.main;
    const bool fork = st.aux[0] && st.aux[1];
    const hipStream_t st_tiny = fork ? st.aux[0] : s;
    const hipStream_t st_chunk = fork ? st.aux[1] : s;
    const int Nc = a.n_nodes > 0 ? a.n_nodes : 1;
    int grid_plan = (Nc + kBlock - 1) / kBlock;
    if (grid_plan > 4 * n_cu) grid_plan = 4 * n_cu;
    hipLaunchKernelGGL(k_preset, dim3(1), dim3(64), 0, s, a.hdr);
    hipLaunchKernelGGL((k_pplan<PS>), dim3(grid_plan), dim3(kBlock), 0, s, a, p);
    hipError_t e = hipGetLastError();
    if (fork && e == hipSuccess) {
        e = hipEventRecord(st.fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(st_tiny, st.fork, 0);
        if (e == hipSuccess) e = hipStreamWaitEvent(st_chunk, st.fork, 0);
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_ptiny<T, PS>), dim3(n_cu * 4), dim3(kBlock), 0, st_tiny, a, p);
    hipLaunchKernelGGL((k_ppred<T, PS>), dim3(n_cu * 4), dim3(kBlock), sizeof(PShared), st_chunk, a, p);
    hipLaunchKernelGGL(k_pchunkscan, dim3(1), dim3(kBlock), 0, st_chunk, a);
    hipLaunchKernelGGL(k_pscatter, dim3(n_cu * 4), dim3(kBlock), sizeof(PShared), st_chunk, a);
    hipLaunchKernelGGL((k_psmall<T, PS>), dim3(n_cu * 4), dim3(kBlock), sizeof(PShared), s, a, p);
    e = hipGetLastError();
    if (fork && e == hipSuccess) {
        e = hipEventRecord(st.join[0], st_tiny);
        if (e == hipSuccess) e = hipEventRecord(st.join[1], st_chunk);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, st.join[0], 0);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, st.join[1], 0);
    }
    return e;
}

size_t part_workspace(int64_t n_nodes, int64_t n_samples) {
    int64_t items = n_samples / kPartMax + n_samples / (kPartMax + 1) + 2;
    size_t o = 256;                                                   // header
    o += (size_t)(items + n_nodes + 1) * sizeof(int4);                // items + small list
    o = (o + 255) & ~(size_t)255;
    o += (size_t)items * sizeof(int32_t);                             // left count per chunk
    o = (o + 255) & ~(size_t)255;
    o += (size_t)(items + 1) * sizeof(int64_t);                       // their exclusive prefix
    o = (o + 255) & ~(size_t)255;
    o += (size_t)items * kWordsPerChunk * sizeof(uint64_t);
    return (o + 255) & ~(size_t)255;
}

void part_bind(int64_t n_nodes, int64_t n_samples, void* ws, PartArgs* a) {
    int64_t items = n_samples / kPartMax + n_samples / (kPartMax + 1) + 2;
    char* b = (char*)ws;
    a->hdr = (int32_t*)b;
    size_t o = 256;
    a->big_items = (int4*)(b + o);
    o += (size_t)(items + n_nodes + 1) * sizeof(int4);
    o = (o + 255) & ~(size_t)255;
    a->chunk_left = (int32_t*)(b + o);
    o += (size_t)items * sizeof(int32_t);
    o = (o + 255) & ~(size_t)255;
    a->chunk_pre = (int64_t*)(b + o);
    o += (size_t)(items + 1) * sizeof(int64_t);
    o = (o + 255) & ~(size_t)255;
    a->pred_bits = (uint64_t*)(b + o);
    a->cap_items = items;
}

hipError_t launch_partition_csr(const PartArgs& a, const ProjCSR& p, int n_cu, const FindStreams& st) {
    if (a.dtype == SOF_F16) return launch_part_t<_Float16>(a, p, n_cu, st);
    return launch_part_t<float>(a, p, n_cu, st);
}
hipError_t launch_partition_hash(const PartArgs& a, const ProjHash& p, int n_cu, const FindStreams& st) {
    if (a.dtype == SOF_F16) return launch_part_t<_Float16>(a, p, n_cu, st);
    return launch_part_t<float>(a, p, n_cu, st);
}

}  // namespace sof

// ---------------------------------------------------------------------------
// C ABI

using namespace sof;

extern "C" int sof_partition(sof_ctx* ctx, const sof_data* data, const sof_frontier* fr,
                             const sof_proj* proj, const sof_params* params, const sof_split* splits,
                             int32_t* out_idx, int32_t* child_offsets, void* ws, size_t ws_bytes,
                             void* stream) {
    if (!ctx) return fail(SOF_ERR_INVALID_ARG, "ctx is NULL");
    int rc;
    if ((rc = check_data(data)) || (rc = check_frontier(fr)) || (rc = check_proj(proj, data)) ||
        (rc = check_params(params)))
        return rc;
    if (!child_offsets) return fail(SOF_ERR_INVALID_ARG, "child_offsets is NULL");
    if (fr->n_nodes > 0 && !splits) return fail(SOF_ERR_INVALID_ARG, "splits is NULL");
    if (fr->n_samples > 0 && !out_idx) return fail(SOF_ERR_INVALID_ARG, "out_idx is NULL");
    if (fr->n_samples > 0 && out_idx == fr->sample_idx)
        return fail(SOF_ERR_INVALID_ARG, "out_idx must not alias sample_idx");
    size_t need = part_workspace(fr->n_nodes, fr->n_samples);
    if ((rc = check_ws_public(ws, ws_bytes, need))) return rc;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    PartArgs a;
    memset(&a, 0, sizeof(a));
    a.x = data->x;
    a.ld = data->ld;
    a.n_rows = data->n_rows;
    a.n_features = data->n_features;
    a.dtype = data->dtype;
    a.node_offsets = fr->node_offsets;
    a.sample_idx = fr->sample_idx;
    a.n_samples = fr->n_samples;
    a.n_nodes = fr->n_nodes;
    a.node_bins = params->node_bins;
    a.bins = params->bins;
    a.splits = splits;
    a.out_idx = out_idx;
    a.child_offsets = child_offsets;
    part_bind(fr->n_nodes, fr->n_samples, ws, &a);
    ProjCSR p{proj->proj_offsets, proj->nz_offsets, proj->nz_feature, proj->nz_weight, proj->n_proj,
              proj->n_nz, proj->nz_value};
    {
        std::lock_guard<std::mutex> g(ctx->launch_mu);
        e = launch_partition_csr(a, p, ctx->n_cu, find_streams(ctx, (hipStream_t)stream));
    }
    if (e != hipSuccess) return hip_fail(e, "partition launch");
    return SOF_OK;
}
