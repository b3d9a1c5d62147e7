// k_find.hip -- batched split search over a whole frontier (paper section 4,
// steps 1-3; section 4.1 for the per-node choice between histograms and
// sorting; section 6 names batching many nodes into one GPU launch as the
// next step, which is what this launch sequence does).
//
// Launch sequence.  Every kernel reads its work counts from device memory,
// so the sequence is graph-capturable.  The plan runs on the caller's stream;
// then the big-node chain, the large mid nodes with the sort blocks, and the
// mid and small nodes run on three streams at once (the size classes are
// independent), and k_reduce runs after they join:
//   k_reset    zero the queue counters
//   k_plan     classify nodes by path and size, allocate queue entries; a
//              small node's item carries its sample range, projection count
//              and first projection index
//   k_expand   write the items of the per-projection and per-group queues
//              (a mid item is self-contained, like a small one)
//   k_brange   big nodes: range of every (projection, chunk); one wave each
//   k_bmerge   big nodes: range of every projection over its chunks
//   k_bhist    big nodes: histogram of every (projection, chunk); one wave each
//   k_bscan    big nodes: chunk histograms summed, boundary scan
//   k_mid      histogram nodes of 513..8192 samples: one block per (node, group of 4
//              projections); one instance up to 4096 samples, one above
//   k_small    histogram nodes up to 512 samples and sort nodes up to 64:
//              one block per node, one wave per projection
//   k_sortblk  sort nodes of 65..8192 samples: bitonic sort in LDS
//   k_reduce   best projection per node for nodes with per-projection slots
// Partial ranges of big nodes go to distinct workspace entries and are merged
// by the next kernel; their chunk histograms are added into per-projection
// histograms with integer atomics (order-free, so the sums are exact).  No
// kernel waits on another block.
#include "sof_device.h"
#include "sof_internal.h"
#include "sof_sampler.h"

namespace sof {

enum { CAT_NONE = 0, CAT_NOSPLIT, CAT_SMALL, CAT_MID, CAT_MID2, CAT_SB, CAT_BIG };

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int64_t clamp64(int64_t x, int64_t lo, int64_t hi) {
    return x < lo ? lo : (x > hi ? hi : x);
}

__device__ __forceinline__ int n_nodes_of(const FindArgs& A) {
    if (!A.n_nodes_dev) return A.n_nodes;
    int n = *A.n_nodes_dev;
    return n < 0 ? 0 : (n > A.n_nodes ? A.n_nodes : n);
}

__device__ __forceinline__ void node_range(const FindArgs& A, int v, int64_t& s0, int64_t& n) {
    int64_t a = clamp64(A.node_offsets[v], 0, A.n_samples);
    int64_t b = clamp64(A.node_offsets[v + 1], a, A.n_samples);
    s0 = a;
    n = b - a;
}

__device__ __forceinline__ int node_bins(const FindArgs& A, int v) {
    if (!A.node_bins) return A.bins;
    int b = A.node_bins[v];
    return b < 2 ? 2 : (b > A.bins ? A.bins : b);
}

__device__ __forceinline__ int row_of(const FindArgs& A, int64_t at) {
    uint32_t r = (uint32_t)A.sample_idx[at];
    return r < (uint32_t)A.n_rows ? (int)r : 0;
}

__device__ __forceinline__ int label_of(const FindArgs& A, int row) {
    uint32_t c = (uint32_t)A.y[row];
    return c < (uint32_t)A.n_classes ? (int)c : 0;
}

// ---------------------------------------------------------------------------
// projection sources

__device__ __forceinline__ int proj_count(const ProjCSR& P, int v) {
    int a = (int)clamp64(P.proj_offsets[v], 0, P.n_proj);
    int b = (int)clamp64(P.proj_offsets[v + 1], a, P.n_proj);
    return b - a;
}
__device__ __forceinline__ int proj_global(const ProjCSR& P, int v, int p) {
    return (int)clamp64(P.proj_offsets[v], 0, P.n_proj) + p;
}
__device__ __forceinline__ int proj_nnz(const ProjCSR& P, int v, int p, int) {
    const int q = proj_global(P, v, p);
    const int64_t j0 = clamp64(P.nz_offsets[q], 0, P.n_nz);
    const int64_t j1 = clamp64(P.nz_offsets[q + 1], j0, P.n_nz);
    return j1 - j0 > SOF_MAX_NNZ ? SOF_MAX_NNZ : (int)(j1 - j0);
}
// Stage the nonzeros of node-local projection p into per-wave LDS (called by
// a whole wave).  Returns z.
__device__ __forceinline__ int proj_stage(const ProjCSR& P, int v, int p, int d, int32_t* lf,
                                          uint32_t* ls) {
    int q = proj_global(P, v, p);
    int64_t j0 = clamp64(P.nz_offsets[q], 0, P.n_nz);
    int64_t j1 = clamp64(P.nz_offsets[q + 1], j0, P.n_nz);
    if (j1 - j0 > SOF_MAX_NNZ) j1 = j0 + SOF_MAX_NNZ;
    int z = (int)(j1 - j0);
    int lane = lane_id();
    if (lane < z) {
        uint32_t f = (uint32_t)P.nz_feature[j0 + lane];
        lf[lane] = f < (uint32_t)d ? (int)f : 0;
        ls[lane] = csr_weight_bits(P, j0 + lane);
    }
    wave_sync();
    return z;
}

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the c-th output of the
// stream started at `seed`.
__device__ __forceinline__ uint64_t splitmix_at(uint64_t seed, uint64_t c) {
    uint64_t z = seed + c * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ int proj_count(const ProjHash& P, int) { return P.k; }
__device__ __forceinline__ SampSpec samp_spec(const ProjHash& P, int d) {
    return SampSpec{P.seed, d, P.z, P.mode, P.wmode};
}
__device__ __forceinline__ int proj_global(const ProjHash& P, int v, int p) { return v * P.k + p; }
__device__ __forceinline__ int proj_nnz(const ProjHash& P, int v, int p, int d) {
    return samp_nnz(samp_spec(P, d), P.tree_of[v], *P.level, P.pos_of[v], p);
}
// The drawn projection staged into per-wave LDS, features ascending (called
// by a whole wave).  Returns z.
__device__ __forceinline__ int proj_stage(const ProjHash& P, int v, int p, int d, int32_t* lf,
                                          uint32_t* ls) {
    const int lane = lane_id();
    const SampSpec sp = samp_spec(P, d);
    const int tree = P.tree_of[v], pos = P.pos_of[v], level = *P.level;
    const int z = __builtin_amdgcn_readfirstlane(samp_nnz(sp, tree, level, pos, p));
    int mine, rank;
    samp_wave(sp, z, tree, level, pos, p, mine, rank);
    if (lane < z) {
        lf[rank] = mine;
        ls[rank] = samp_weight_bits(sp, tree, level, pos, p, rank);
    }
    wave_sync();
    return z;
}

// index of node-local projection p in the call, given the node's first (q0)
__device__ __forceinline__ int item_q(const ProjCSR&, int, int q0, int p) { return q0 + p; }
__device__ __forceinline__ int item_q(const ProjHash& P, int v, int, int p) { return v * P.k + p; }
// Key of the random-width bins of node-local projection p: the projection's
// index in the call for given projections, and for drawn ones the sampler's
// counter of (tree, level, position, projection) without its draw field, so
// that a node's bins depend on its tree position only (batched trees equal
// single-tree runs)
__device__ __forceinline__ uint64_t bin_key(const ProjCSR&, int, int q0, int p) { return (uint64_t)(q0 + p); }
__device__ __forceinline__ uint64_t bin_key(const ProjHash& P, int v, int, int p) {
    return samp_counter(P.tree_of[v], *P.level, P.pos_of[v], p, 0) >> 4;
}

// ---------------------------------------------------------------------------
// allocation helpers

__device__ __forceinline__ int block_dequeue(int32_t* ctr, int* s_item) {
    __syncthreads();
    if (threadIdx.x == 0) *s_item = atomicAdd(ctr, 1);
    __syncthreads();
    return *s_item;
}

__device__ __forceinline__ int count_of(const FindArgs& A, int h, int64_t cap) {
    int c = A.ws.hdr[h];
    return (int)(c < 0 ? 0 : (c > cap ? cap : c));
}

__device__ __forceinline__ void write_nosplit(const FindArgs& A, int v, int kind, int64_t n) {
    SplitRec* o = (SplitRec*)A.out + v;
    SplitRec r;
    r.proj = -1; r.kind = kind; r.bin = -1; r.threshold = 0.f; r.lo = 0.f; r.scale = 0.f;
    r.n_left = (int32_t)n; r.n_right = 0; r.flags = 0; r.gain = 0.f;
    *o = r;
}

// hist_out row of global projection q from a count accessor (lanes of one wave)
template <class H>
__device__ __forceinline__ void write_hist_row(const FindArgs& A, int q, const H& h, int B) {
    if (!A.hist_out) return;
    const int C = A.n_classes, Bm = A.bins;
    int32_t* row = A.hist_out + (int64_t)q * Bm * C;
    for (int e = lane_id(); e < Bm * C; e += kWave) {
        int b = e / C, c = e - b * C;
        row[e] = b < B ? (int32_t)h(b, c) : 0;
    }
}
__device__ __forceinline__ void write_zero_row(const FindArgs& A, int q) {
    if (!A.hist_out) return;
    const int n = A.bins * A.n_classes;
    int32_t* row = A.hist_out + (int64_t)q * n;
    for (int e = lane_id(); e < n; e += kWave) row[e] = 0;
}

// Histogram accessor over a wave's class-major LDS histogram h[c * Bs + b]
// (Bs a multiple of 4, bins B..Bs-1 zero): h(b, c) is the count of class c in
// bin b; load4/store4 move bins b0..b0+3 of class c as one 16-byte access.
// The boundary scan overwrites the counts with left counts (prefix sums).
struct LdsHistCM {
    int32_t* h;
    int Bs;
    __device__ uint32_t operator()(int b, int c) const { return (uint32_t)h[c * Bs + b]; }
    __device__ uint4 load4(int b0, int c) const { return *(const uint4*)(h + c * Bs + b0); }
    __device__ void store4(int b0, int c, uint4 v) const { *(uint4*)(h + c * Bs + b0) = v; }
};

__host__ __device__ constexpr int bins_stride(int bins) { return (bins + 3) & ~3; }

// ---------------------------------------------------------------------------
// boundary scans (one wave)

// Histogram path, screened scan by one wave over a class-major histogram
// (lane l owns bins 4l..4l+3; B <= 256).  Class by class, an integer prefix
// over the wave gives every boundary's left count, which is written back over
// the counts in place.
//
// Screening: every boundary after a non-empty bin gets an FP32 score
// q = S_L / n_L + S_R / n_R.  Counts below 2^24 are exact in FP32, so only
// the C fused squares-and-adds, the two reciprocals (1 ulp each) and the
// final product and sum round: |q - Q| <= (C + 4) 2^-24 Q <= 20 * 2^-24 Q
// for C <= 16.  Any boundary whose exact Q could reach the largest then scores
// at least qmax (1 - 2^-16).  Those contenders (usually one) are evaluated
// exactly from their integer left counts (lane c reads class c's from LDS)
// and compared as N1 D2 > N2 D1 in 128 bits, ties to the lower bin.  A
// boundary after an empty bin repeats the previous boundary's counts, so it
// can never win under that tie rule and is skipped.  pc: 16 ints of wave
// scratch in LDS (the node's class totals).
constexpr float kScreenKeep = 1.0f - 1.0f / 65536.0f;
// When more than kSerialContenders boundaries pass that screen (a flat score
// curve: many samples and a projection that separates the classes little),
// they are screened again in binary64, one lane per boundary: with the class
// left counts exact, S_L, S_R < 2^48 and n_L, n_R are exact in binary64, and
// Q64 = S_L / n_L + S_R / n_R (two correctly rounded divisions, one sum) lies
// within 2 * 2^-53 Q of Q.  Every boundary whose exact Q is the largest then
// scores at least max Q64 (1 - 2^-48); only those reach the exact comparison.
// PRE = false leaves this stage out (the small-node kernel with random-width
// bins, whose register budget it would overflow).
constexpr int kSerialContenders = 4;

// qfloor (optional): the FP32 score of the caller's incumbent from an earlier
// scan.  When this scan's best score is below qfloor (1 - 2^-16), its exact
// best Q is below the incumbent's (both scores are within 20 * 2^-24 of their
// exact values), so it cannot win or tie and is returned invalid without its
// exact evaluation.  qmax_out (optional) receives this scan's best score.
template <bool PRE = true>
__device__ Cand scan_hist_fast(const LdsHistCM& h, int B, int C, int64_t n, float lo, float scale, int32_t* pc,
                               float qfloor = -1.f, float* qmax_out = nullptr) {
    const int lane = lane_id();
    const int b0 = lane * 4;
    const float nf = (float)n;
    float nL[4] = {0.f, 0.f, 0.f, 0.f}, SL[4] = {0.f, 0.f, 0.f, 0.f}, SR[4] = {0.f, 0.f, 0.f, 0.f};
    uint32_t filled = 0;
    uint64_t SP = 0;
    for (int c = 0; c < C; ++c) {
        uint4 q4 = make_uint4(0u, 0u, 0u, 0u);
        if (b0 < B) q4 = h.load4(b0, c);
        const uint32_t s0 = q4.x, s1 = s0 + q4.y, s2 = s1 + q4.z, s3 = s2 + q4.w;
        const uint32_t incl = wave_scan_u(s3);
        const uint32_t excl = incl - s3;
        const uint32_t Pi = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        SP += (uint64_t)Pi * Pi;
        if (lane == 0) pc[c] = (int32_t)Pi;
        const uint32_t li[4] = {excl + s0, excl + s1, excl + s2, excl + s3};
        if (b0 < B) h.store4(b0, c, make_uint4(li[0], li[1], li[2], li[3]));
        const uint32_t hv[4] = {q4.x, q4.y, q4.z, q4.w};
        const float Pf = (float)Pi;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float l = (float)li[i];
            const float r = Pf - l;
            nL[i] += l;
            SL[i] = __fmaf_rn(l, l, SL[i]);
            SR[i] = __fmaf_rn(r, r, SR[i]);
            if (hv[i] != 0) filled |= 1u << i;
        }
    }
    float q[4];
    float qb = -1.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const bool ok = b0 + i < B - 1 && ((filled >> i) & 1u) && nL[i] < nf;
        q[i] = ok ? SL[i] * __builtin_amdgcn_rcpf(nL[i]) + SR[i] * __builtin_amdgcn_rcpf(nf - nL[i]) : -1.f;
        qb = fmaxf(qb, q[i]);
    }
    const float qmax = wave_max_f(qb);
    if (qmax_out) *qmax_out = qmax;
    Cand best;
    cand_invalid(best);
    best.SP = SP;
    best.lo = lo;
    best.scale = scale;
    if (!(qmax >= 0.f)) return best;
    if (qmax < qfloor * kScreenKeep) return best;
    const float keep = qmax * kScreenKeep;
    wave_sync();   // pc[] and the left counts written above are read by other lanes below
    const uint32_t pcv = lane < C ? (uint32_t)pc[lane] : 0u;
    uint32_t cm = 0;   // this lane's contenders (bit i: boundary after bin b0 + i)
    int ncont = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (q[i] >= 0.f && q[i] >= keep) cm |= 1u << i;
        ncont += __popcll(__ballot((cm >> i) & 1u));
    }
    if (PRE && ncont > kSerialContenders) {
        // Q64 of the lane's boundary b0 + i, recomputed in the second pass
        // (the same operations, so the same value) rather than kept
        auto q64 = [&](int i) -> double {
            uint64_t nLx = 0, SLx = 0, SRx = 0;
            for (int c = 0; c < C; ++c) {
                const uint64_t lc = h(b0 + i, c);
                const uint64_t rc = (uint64_t)(uint32_t)pc[c] - lc;
                nLx += lc;
                SLx += lc * lc;
                SRx += rc * rc;
            }
            return (double)SLx / (double)nLx + (double)SRx / (double)((uint64_t)n - nLx);
        };
        double qdb = -1.0;
        for (uint32_t t = cm; t; t &= t - 1) qdb = fmax(qdb, q64(__builtin_ctz(t)));
        const double keepd = wave_max_d(qdb) * (1.0 - 0x1p-48);
        for (uint32_t t = cm; t; t &= t - 1) {
            const int i = __builtin_ctz(t);
            if (q64(i) < keepd) cm &= ~(1u << i);
        }
    }
    bool have = false;
    u128 bN = 0;
    uint64_t bD = 0, bSL = 0, bSR = 0;
    int bb = 0;
    uint32_t bnL = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint64_t m = __ballot((cm >> i) & 1u);
        while (m) {
            const int ln = __builtin_ctzll(m);
            m &= m - 1;
            const int b = ln * 4 + i;
            const uint32_t lcv = lane < C ? h(b, lane) : 0u;
            uint32_t nLx = 0;
            uint64_t SLx = 0, SRx = 0;
            for (int c = 0; c < C; ++c) {
                const uint32_t lc = (uint32_t)__builtin_amdgcn_readlane((int)lcv, c);
                const uint32_t rc = (uint32_t)__builtin_amdgcn_readlane((int)pcv, c) - lc;
                nLx += lc;
                SLx += (uint64_t)lc * lc;
                SRx += (uint64_t)rc * rc;
            }
            u128 N;
            uint64_t D;
            if (!make_q((int64_t)nLx, n - (int64_t)nLx, SLx, SRx, N, D)) continue;
            if (!have || q_greater(N, D, bN, bD) || (!q_greater(bN, bD, N, D) && b < bb)) {
                have = true; bN = N; bD = D; bSL = SLx; bSR = SRx; bb = b; bnL = nLx;
            }
        }
    }
    if (have) {
        best.N = bN;
        best.D = bD;
        best.SL = bSL;
        best.SR = bSR;
        best.pos = bb;
        best.nL = (int32_t)bnL;
        best.nR = (int32_t)(n - (int64_t)bnL);
        best.thr = hist_threshold(lo, scale, bb);
    }
    return best;
}

// Entropy criterion over a class-major histogram (one wave; lane l owns bins
// 4l..4l+3).  Every boundary b (0..B-2) with both sides non-empty gets
// E = sum_c f(l_c) + sum_c f(r_c) - f(n_L) - f(n_R) in binary64, the sums over
// c ascending, with f and the log of sof_device.h (read from the call's table
// of f for counts below its size, which the same function filled, so the
// values are identical either way); the largest E wins, the
// lowest boundary on ties.  The winner is returned with N = key(E), D = 1, so
// the exact comparisons between projections order it by E; SL, SR, SP carry
// the bits of sum f(l_c), sum f(r_c) and sum f(P_c) for the node record.
// k ln k for the entropy scans: the block's LDS copy of its first nl entries,
// then the call's table (ng entries), then the function itself -- the same
// bits from any of the three
struct Flnk {
    const double* lds;
    int64_t nl;
    const double* glob;
    int64_t ng;
};
__device__ __forceinline__ double flnk_at(const Flnk& t, int64_t k) {
    return k < t.nl ? t.lds[k] : (k < t.ng ? t.glob[k] : klnk(k));
}

__device__ Cand scan_hist_entropy(const LdsHistCM& h, int B, int C, int64_t n, float lo, float scale,
                                  const Flnk& tab) {
    const int lane = lane_id();
    const int b0 = lane * 4;
    double FL[4] = {0.0, 0.0, 0.0, 0.0}, FR[4] = {0.0, 0.0, 0.0, 0.0};
    uint32_t nLi[4] = {0u, 0u, 0u, 0u};
    double FP = 0.0;
    for (int c = 0; c < C; ++c) {
        uint4 q4 = make_uint4(0u, 0u, 0u, 0u);
        if (b0 < B) q4 = h.load4(b0, c);
        const uint32_t s0 = q4.x, s1 = s0 + q4.y, s2 = s1 + q4.z, s3 = s2 + q4.w;
        const uint32_t incl = wave_scan_u(s3);
        const uint32_t ex = incl - s3;
        const uint32_t Pi = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        FP = __dadd_rn(FP, flnk_at(tab, Pi));
        const uint32_t li[4] = {ex + s0, ex + s1, ex + s2, ex + s3};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            nLi[i] += li[i];
            FL[i] = __dadd_rn(FL[i], flnk_at(tab, li[i]));
            FR[i] = __dadd_rn(FR[i], flnk_at(tab, Pi - li[i]));
        }
    }
    double bE = 0.0, bFL = 0.0, bFR = 0.0;
    int bi = -1;
    uint32_t bnL = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t nL = nLi[i], nR = n - (int64_t)nLi[i];
        if (b0 + i < B - 1 && nL >= 1 && nR >= 1) {
            const double E = __dsub_rn(__dsub_rn(__dadd_rn(FL[i], FR[i]), flnk_at(tab, nL)),
                                       flnk_at(tab, nR));
            if (bi < 0 || E > bE) { bE = E; bi = i; bFL = FL[i]; bFR = FR[i]; bnL = nLi[i]; }
        }
    }
    Cand best;
    cand_invalid(best);
    best.SP = d_bits(FP);
    best.lo = lo;
    best.scale = scale;
    const int win = wave_best_lane(bi >= 0, (u128)dkey(bE), 1ull, b0 + bi);
    if (win < 0) return best;
    const uint64_t kE = dkey(bE);
    best.N = (u128)(((uint64_t)__builtin_amdgcn_readlane((int)(uint32_t)(kE >> 32), win) << 32) |
                    (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)kE, win));
    best.D = 1;
    const uint64_t fl = d_bits(bFL), fr = d_bits(bFR);
    best.SL = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(fl >> 32), win) << 32) |
              (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)fl, win);
    best.SR = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(fr >> 32), win) << 32) |
              (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)fr, win);
    best.pos = __builtin_amdgcn_readlane(b0 + bi, win);
    best.nL = __builtin_amdgcn_readlane((int)bnL, win);
    best.nR = (int32_t)(n - (int64_t)best.nL);
    best.thr = hist_threshold(lo, scale, best.pos);
    return best;
}

// ---------------------------------------------------------------------------
// Histogram bins of one projection.  Equal width: the closed-form index.
// Random width (bin boundaries at random-width intervals, after the
// Introduction's footnote; the sampling rule is this library's reading): the
// B widths of the call's q-th projection are g_j = 1 + (bits 63..48 of
// SplitMix64 output 256 q + j), G_i = g_0 + ... + g_{i-1} (exact integers,
// G_B <= 2^24), boundary i = 1..B-1 is lo + (G_i / G_B) (hi - lo) with each
// operation rounded once, and a value's bin is the number of boundaries <= v.
//
// Routing without a search over the boundaries: a wave builds, per
// projection, a table over kRwCells equal-width cells of [lo, hi] with lut[c]
// = the number of boundaries whose cell is below c.  The cell index is
// monotone in the value, so a boundary in an earlier cell is < v and one in a
// later cell is > v: bin(v) = lut[c(v)] + the boundaries of cell c(v) that are
// <= v (usually none or one, found by a short binary search).

struct EqualBins {
    float lo, scale;
    int B;
    __device__ int operator()(float v) const { return bin_index(v, lo, scale, B); }
};

constexpr int kRwCells = 511;

struct RwTable {
    float t[256];                  // boundary i+1 at t[i] (i < B-1), +inf above
    int32_t lut[kRwCells + 1];
};

__device__ __forceinline__ float rw_cell_scale(float lo, float hi) {
    float s = __fdiv_rn((float)kRwCells, __fsub_rn(hi, lo));
    return s <= FLT_MAX ? s : FLT_MAX;
}
__device__ __forceinline__ int rw_cell(float x, float lo, float sc) {
    const float t = __fmul_rn(__fsub_rn(x, lo), sc);
    return t < (float)kRwCells ? (int)t : kRwCells - 1;
}
__device__ __forceinline__ uint32_t rw_width(uint64_t seed, uint64_t q, int j) {
    return 1u + (uint32_t)(splitmix_at(seed, (uint64_t)q * 256u + (uint64_t)j) >> 48);
}

// Build projection q's table (one wave, every lane; lane l owns bins 4l..4l+3).
__device__ void rw_build(RwTable& T, uint64_t seed, uint64_t q, int B, float lo, float hi, float sc) {
    const int lane = lane_id();
    uint32_t g[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) g[i] = 4 * lane + i < B ? rw_width(seed, q, 4 * lane + i) : 0u;
    const uint32_t s0 = g[0], s1 = s0 + g[1], s2 = s1 + g[2], s3 = s2 + g[3];
    const uint32_t incl = wave_scan_u(s3);
    const uint32_t ex = incl - s3;
    const float tot = (float)(uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    const float wd = __fsub_rn(hi, lo);
    const uint32_t G[4] = {ex + s0, ex + s1, ex + s2, ex + s3};   // G_{j+1}, j = 4 lane + i
    float tv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        tv[i] = 4 * lane + i < B - 1 ? __fadd_rn(lo, __fmul_rn(__fdiv_rn((float)G[i], tot), wd)) : INFINITY;
    *(float4*)&T.t[4 * lane] = make_float4(tv[0], tv[1], tv[2], tv[3]);
    *(int4*)&T.lut[8 * lane] = make_int4(0, 0, 0, 0);
    *(int4*)&T.lut[8 * lane + 4] = make_int4(0, 0, 0, 0);
    wave_sync();
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (4 * lane + i < B - 1) atomicAdd(&T.lut[rw_cell(tv[i], lo, sc) + 1], 1);
    wave_sync();
    const int4 a = *(const int4*)&T.lut[8 * lane];
    const int4 b = *(const int4*)&T.lut[8 * lane + 4];
    const uint32_t p0 = a.x, p1 = p0 + a.y, p2 = p1 + a.z, p3 = p2 + a.w;
    const uint32_t p4 = p3 + b.x, p5 = p4 + b.y, p6 = p5 + b.z, p7 = p6 + b.w;
    const uint32_t e8 = wave_scan_u(p7) - p7;
    *(int4*)&T.lut[8 * lane] = make_int4(e8 + p0, e8 + p1, e8 + p2, e8 + p3);
    *(int4*)&T.lut[8 * lane + 4] = make_int4(e8 + p4, e8 + p5, e8 + p6, e8 + p7);
    wave_sync();
}

struct RwBins {
    const RwTable* T;
    float lo, sc;
    __device__ int operator()(float v) const {
        const int c = rw_cell(v, lo, sc);
        int a = T->lut[c], b = T->lut[c + 1];
        while (a < b) {
            const int m = (a + b) >> 1;
            if (T->t[m] <= v) a = m + 1;
            else b = m;
        }
        return a;
    }
};

// Boundary b+1 of projection q (the random-width split threshold: bin(v) <= b
// iff v < it), by one wave with uniform loop bounds.
__device__ float rw_boundary(uint64_t seed, uint64_t q, int B, float lo, float hi, int b) {
    const int lane = lane_id();
    uint32_t gb = 0, gt = 0;
    for (int j0 = 0; j0 < 256; j0 += kWave) {
        const int j = j0 + lane;
        if (j < B) {
            const uint32_t g = rw_width(seed, q, j);
            gt += g;
            if (j <= b) gb += g;
        }
    }
    const uint32_t Gb = wave_sum_u(gb), GB = wave_sum_u(gt);
    return __fadd_rn(lo, __fmul_rn(__fdiv_rn((float)Gb, (float)GB), __fsub_rn(hi, lo)));
}

// a better than b, ties to the lower projection
__device__ __forceinline__ bool cand_better_proj(const Cand& a, const Cand& b) {
    if (a.D == 0) return false;
    if (b.D == 0) return true;
    if (q_greater(a.N, a.D, b.N, b.D)) return true;
    if (q_greater(b.N, b.D, a.N, a.D)) return false;
    return a.proj < b.proj;
}

// ---------------------------------------------------------------------------
// shared memory of the persistent block kernels

struct WaveScratch {
    int32_t lf[16];
    uint32_t ls[16];
    int32_t pc[16];
    int32_t pcs[16];      // parent counts written by the histogram scan
    int32_t bz[8];        // small nodes: nonzeros of the staged batch of projections
    int32_t blf[8 * 16];  // ... their feature ids (16 per projection)
    uint32_t bls[8 * 16]; // ... and sign masks
    float red[2];
    int32_t pad[2];
    Cand best;
    uint32_t sk[kWave];   // sort path of small nodes: keys, then sorted keys
    int32_t sl[kWave];    // sorted labels
};

constexpr int kMidGroup = kWavesPerBlock;   // projections of one mid-node item

struct BlockShared {
    int item;
    int pad[3];
    float lo[kWavesPerBlock];
    float hi[kWavesPerBlock];
    float glo[kMidGroup][kWavesPerBlock];   // mid items: range of projection j seen by wave w
    float ghi[kMidGroup][kWavesPerBlock];
    int32_t gz[kMidGroup];                  // mid items: nonzeros of projection j
    int32_t gpad[4 - kMidGroup % 4];
    WaveScratch w[kWavesPerBlock];
};

// entropy launches: k ln k for k = 0 .. 1024 in LDS (every count of a small
// node, the common counts of a mid node)
constexpr int kFlnkLds = 1025;

size_t find_smem_main(int bins, int classes, bool random_bins, bool entropy) {
    return sizeof(BlockShared) + (size_t)kWavesPerBlock * bins_stride(bins) * classes * sizeof(int32_t) +
           (random_bins ? (size_t)kWavesPerBlock * sizeof(RwTable) : 0) +
           (entropy ? (size_t)kFlnkLds * sizeof(double) : 0);
}

__device__ __forceinline__ BlockShared& block_shared(char* smem) { return *(BlockShared*)smem; }
__device__ __forceinline__ int32_t* wave_hist(char* smem, int w, int bins, int C) {
    return (int32_t*)(smem + sizeof(BlockShared)) + (size_t)w * bins_stride(bins) * C;
}
// the wave's random-width table (launches with random-width bins only)
__device__ __forceinline__ RwTable& wave_rw(char* smem, int w, int bins, int C) {
    return ((RwTable*)(smem + sizeof(BlockShared) + (size_t)kWavesPerBlock * bins_stride(bins) * C * sizeof(int32_t)))[w];
}
static_assert(sizeof(BlockShared) % 8 == 0 && sizeof(RwTable) % 8 == 0, "the k ln k copy is 8-byte aligned");
// the block's copy of k ln k, k = 0 .. kFlnkLds - 1 (entropy launches only)
__device__ __forceinline__ double* block_flnk(char* smem, int bins, int C, bool rw) {
    return (double*)(smem + sizeof(BlockShared) + (size_t)kWavesPerBlock * bins_stride(bins) * C * sizeof(int32_t) +
                     (rw ? (size_t)kWavesPerBlock * sizeof(RwTable) : 0));
}
template <bool RW>
__device__ __forceinline__ void fill_flnk(const FindArgs& A, char* smem) {
    double* t = block_flnk(smem, A.bins, A.n_classes, RW);
    for (int i = threadIdx.x; i < kFlnkLds; i += kBlock) t[i] = i < A.ws.cap_flnk ? A.ws.flnk[i] : klnk(i);
}

// block-wide min/max of per-thread values (all threads call)
__device__ __forceinline__ void block_minmax(BlockShared& S, float& lo, float& hi) {
    const int w = threadIdx.x >> 6;
    lo = wave_min(lo);
    hi = wave_max(hi);
    if (lane_id() == 0) { S.lo[w] = lo; S.hi[w] = hi; }
    __syncthreads();
    lo = fminf(fminf(S.lo[0], S.lo[1]), fminf(S.lo[2], S.lo[3]));
    hi = fmaxf(fmaxf(S.hi[0], S.hi[1]), fmaxf(S.hi[2], S.hi[3]));
}

// Sort path for n <= 64 (one wave; lane i < n holds sample i's value and
// label).  Each lane ranks its order-preserving key against all n keys in LDS
// (ties by lane), scatters (key, label) to its rank, then per-class inclusive
// scans over the sorted labels give the left counts at every sorted
// position.  Boundaries only between distinct values.
// ENT: the entropy criterion at every boundary between distinct values,
// E = ((sum_c f(l_c) + sum_c f(r_c)) - f(n_L)) - f(n_R) in binary64 with the
// class sums ascending (f from tab), ordered through key(E) with D = 1 as in
// the histogram scan; SL, SR, SP carry the bits of the three class sums.
template <bool ENT>
__device__ Cand scan_sort_small(WaveScratch& WS, float val, int lab, int64_t n, int C, const Flnk& tab) {
    const int lane = lane_id();
    const bool real = lane < n;
    const uint32_t key = fkey(val);
    if (real) WS.sk[lane] = key;
    wave_sync();
    int rank = 0;
    for (int j = 0; j < n; ++j) {
        const uint32_t kj = WS.sk[j];
        rank += (kj < key || (kj == key && j < lane)) ? 1 : 0;
    }
    wave_sync();
    if (real) {
        WS.sk[rank] = key;
        WS.sl[rank] = lab;
    }
    wave_sync();
    const uint32_t myk = real ? WS.sk[lane] : 0xffffffffu;
    const int mylab = real ? WS.sl[lane] : -1;
    const uint32_t nextk = lane + 1 < n ? WS.sk[lane + 1] : 0xffffffffu;
    const uint32_t k0 = WS.sk[0];
    wave_sync();
    uint64_t SL = 0, SR = 0, SP = 0;
    double FL = 0.0, FR = 0.0, FP = 0.0;
    for (int c = 0; c < C; ++c) {
        const uint32_t l = wave_incl_scan((real && mylab == c) ? 1u : 0u);
        const uint32_t Pc = (uint32_t)WS.pc[c];
        const uint32_t r = Pc - l;
        if (ENT) {
            FL = __dadd_rn(FL, flnk_at(tab, l));
            FR = __dadd_rn(FR, flnk_at(tab, r));
            FP = __dadd_rn(FP, flnk_at(tab, Pc));
        } else {
            SL += (uint64_t)l * l;
            SR += (uint64_t)r * r;
            SP += (uint64_t)Pc * Pc;
        }
    }
    u128 N = 0;
    uint64_t D = 0;
    bool ok = lane + 1 < n && myk < nextk;
    if (ENT) {
        const double E = __dsub_rn(__dsub_rn(__dadd_rn(FL, FR), flnk_at(tab, lane + 1)),
                                   flnk_at(tab, n - (int64_t)lane - 1));
        N = (u128)dkey(E);
        D = 1;
        SL = d_bits(FL);
        SR = d_bits(FR);
        SP = d_bits(FP);
    } else {
        ok = ok && make_q((int64_t)lane + 1, n - (int64_t)lane - 1, SL, SR, N, D);
    }
    const int win = wave_best_lane(ok, N, D, lane);
    Cand c;
    cand_invalid(c);
    c.SP = SP;
    c.lo = kfloat(k0);
    if (win >= 0) {
        const uint64_t nlo = __shfl((uint64_t)N, win), nhi = __shfl((uint64_t)(N >> 64), win);
        c.N = ((u128)nhi << 64) | nlo;
        c.D = __shfl(D, win);
        c.SL = __shfl(SL, win);
        c.SR = __shfl(SR, win);
        c.pos = win;
        c.nL = win + 1;
        c.nR = (int32_t)(n - c.nL);
        c.thr = kfloat(__shfl(myk, win));
        c.scale = 0.f;
    }
    return c;
}

// ---------------------------------------------------------------------------
// Row loads shared by the small and mid nodes.  A thread holds R samples
// (sample t + r * stride in slot r).  Slots past the node's end repeat its
// last sample (row 0 for an empty node), so every address is valid and the
// loads of one column are issued together, without a branch per slot; those
// slots are masked out of the range and the histogram by `lab < 0` (small)
// or by the sample index (mid).  Columns are addressed as a uniform base plus
// a 32-bit byte offset per slot (row ids are below 2^30).

template <typename T>
__device__ __forceinline__ float ldx_off(const T* col, uint32_t off) {
    // keep the offset a 32-bit register at each load: otherwise the compiler
    // hoists its widening out of the column loop and holds a 64-bit copy of
    // every slot's offset across the whole projection
    asm volatile("" : "+v"(off));
    return ldx((const T*)((const char*)col + off), 0);
}

// v[r] = sum over the projection's z nonzeros (lf/ls, CSR order) of
// +/- x[f][row r].  FB columns are requested per round trip; when fewer than
// FB remain, the spare requests read the first column of the batch (a valid
// address) and are not added.  Adds stay in CSR order.
template <typename T, int R, int FB = 1>
__device__ __forceinline__ void gather_rows(const FindArgs& A, const int32_t* lf, const uint32_t* ls, int z,
                                            const uint32_t (&off)[R], float (&val)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) val[r] = 0.f;
    for (int j = 0; j < z; j += FB) {
        const int nf = z - j < FB ? z - j : FB;
        float x[FB][R];
        uint32_t sg[FB];
#pragma unroll
        for (int t = 0; t < FB; ++t) {
            const int jt = t < nf ? j + t : j;
            const int f = __builtin_amdgcn_readfirstlane(lf[jt]);
            sg[t] = __builtin_amdgcn_readfirstlane(ls[jt]);
            const T* col = (const T*)A.x + (int64_t)f * A.ld;
#pragma unroll
            for (int r = 0; r < R; ++r) x[t][r] = ldx_off(col, off[r]);
        }
#pragma unroll
        for (int t = 0; t < FB; ++t) {
            if (t >= nf) break;
#pragma unroll
            for (int r = 0; r < R; ++r) val[r] = __fadd_rn(val[r], weighted_term(x[t][r], sg[t]));
        }
    }
}

// ---------------------------------------------------------------------------
// Small nodes stage the nonzeros of a batch of kSmallBatch projections
// (p0, p0 + pstep, ...; those >= k get none) into the wave's scratch in two
// phases: batch_range (lane g reads projection g's CSR range) and batch_fill
// (every lane fetches two of the batch's 128 (projection, nonzero) slots), so
// a caller can issue its own loads between them.  Every index is clamped into
// its array.

constexpr int kSmallBatch = 8;

// The CSR ranges of a batch (lane g < kSmallBatch: projection p0 + pstep g,
// index q0 + p in the call), requested before the caller's other loads;
// batch_fill then stages the nonzeros.
struct BatchRange {
    int64_t a;
    int cnt;
};
__device__ __forceinline__ BatchRange batch_range(const ProjCSR& P, int q0, int p0, int pstep, int k) {
    const int lane = lane_id();
    BatchRange r{0, 0};
    if (lane < kSmallBatch) {
        const int p = p0 + pstep * lane;
        if (p < k) {
            int q = q0 + p;
            q = q < P.n_proj ? (q < 0 ? 0 : q) : P.n_proj - 1;
            r.a = clamp64(P.nz_offsets[q], 0, P.n_nz);
            const int64_t b = clamp64(P.nz_offsets[q + 1], r.a, P.n_nz);
            r.cnt = (int)(b - r.a > SOF_MAX_NNZ ? SOF_MAX_NNZ : b - r.a);
        }
    }
    return r;
}
__device__ __forceinline__ BatchRange batch_range(const ProjHash&, int, int, int, int) { return BatchRange{0, 0}; }
__device__ __forceinline__ void batch_fill(const ProjCSR& P, BatchRange r, int, int, int, int, int d,
                                           WaveScratch& WS) {
    const int lane = lane_id();
    const int64_t a = r.a;
    const int cnt = r.cnt;
    if (lane < kSmallBatch) WS.bz[lane] = cnt;
#pragma unroll
    for (int i = 0; i < kSmallBatch * SOF_MAX_NNZ / kWave; ++i) {
        const int e = lane + kWave * i;
        const int g = e / SOF_MAX_NNZ, t = e % SOF_MAX_NNZ;
        const int64_t ag = __shfl(a, g);
        const int cg = __shfl(cnt, g);
        if (t < cg) {
            const uint32_t f = (uint32_t)P.nz_feature[ag + t];
            WS.blf[e] = f < (uint32_t)d ? (int)f : 0;
            WS.bls[e] = csr_weight_bits(P, ag + t);
        }
    }
    wave_sync();
}
__device__ __forceinline__ void batch_fill(const ProjHash& P, BatchRange, int v, int p0, int pstep, int k, int d,
                                           WaveScratch& WS) {
    for (int g = 0; g < kSmallBatch; ++g) {
        const int p = p0 + pstep * g;
        int z = 0;
        if (p < k) z = proj_stage(P, v, p, d, WS.blf + SOF_MAX_NNZ * g, WS.bls + SOF_MAX_NNZ * g);
        if (lane_id() == 0) WS.bz[g] = z;
    }
    wave_sync();
}

// ---------------------------------------------------------------------------
// small nodes: one block per node, wave w takes projections w, w+4, ...

constexpr int kSmallR = kSmallMax / kWave;   // up to 8 samples per lane

template <typename T, class PS, int R, bool RW, bool ENT>
__device__ void do_small_r(const FindArgs& A, const PS& P, int v, int64_t s0, int64_t n, int k, int q0,
                           char* smem) {
    BlockShared& S = block_shared(smem);
    const int w = threadIdx.x >> 6, lane = lane_id();
    const int C = A.n_classes, Bm = A.bins;
    const int B = node_bins(A, v);
    const bool sortp = n < A.sort_threshold;
    WaveScratch& WS = S.w[w];
    int32_t* hist = wave_hist(smem, w, Bm, C);

    // row ids and the first batch's CSR ranges together, then labels and the
    // batch's nonzeros
    uint32_t rid[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = lane + (int64_t)r * kWave;
        rid[r] = n > 0 ? (uint32_t)A.sample_idx[s0 + (i < n ? i : n - 1)] : 0u;
    }
    BatchRange br{0, 0};
    if (w < k) br = batch_range(P, q0, w, kWavesPerBlock, k);
    uint32_t off[R];
    int lab[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = lane + (int64_t)r * kWave;
        const int row = rid[r] < (uint32_t)A.n_rows ? (int)rid[r] : 0;
        off[r] = (uint32_t)row * (uint32_t)sizeof(T);
        const int y = label_of(A, row);
        lab[r] = i < n ? y : -1;
    }
    if (w < k) batch_fill(P, br, v, w, kWavesPerBlock, k, A.n_features, WS);
    if (lane < 16) WS.pc[lane] = 0;
    wave_sync();
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (lab[r] >= 0) atomicAdd(&WS.pc[lab[r]], 1);
    wave_sync();

    // The wave's running best lives in its LDS slot and is replaced by a plain
    // store: a conditional register copy of the 80-byte candidate was compiled
    // for gfx950 into code that kept the old 128-bit N while taking the other
    // fields of the new candidate.
    if (lane == 0) cand_invalid(WS.best);
    wave_sync();
    float bestq = -1.f;   // the incumbent's FP32 score (Gini histogram scans)
    for (int pb = w; pb < k; pb += kWavesPerBlock * kSmallBatch) {
      if (pb != w) batch_fill(P, batch_range(P, q0, pb, kWavesPerBlock, k), v, pb, kWavesPerBlock, k, A.n_features, WS);
      for (int gi = 0; gi < kSmallBatch; ++gi) {
        const int p = pb + kWavesPerBlock * gi;
        if (p >= k) break;
        const int z = __builtin_amdgcn_readfirstlane(WS.bz[gi]);
        float val[R];
        gather_rows<T, R, 4>(A, WS.blf + SOF_MAX_NNZ * gi, WS.bls + SOF_MAX_NNZ * gi, z, off, val);
        float lo = INFINITY, hi = -INFINITY;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (lab[r] >= 0) { lo = fminf(lo, val[r]); hi = fmaxf(hi, val[r]); }
        lo = wave_min(lo);
        hi = wave_max(hi);
        Cand c;
        if (sortp) {
            c = scan_sort_small<ENT>(WS, val[0], lab[0], n, C,
                                     Flnk{ENT ? block_flnk(smem, Bm, C, RW) : nullptr, ENT ? kFlnkLds : 0, nullptr, 0});
            write_zero_row(A, item_q(P, v, q0, p));
        } else {
            const float scale = bin_scale(B, lo, hi);
            const int Bs = bins_stride(Bm);
            for (int e = lane * 4; e < C * Bs; e += kWave * 4) *(int4*)(hist + e) = make_int4(0, 0, 0, 0);
            wave_sync();
            if (RW) {
                RwTable& tab = wave_rw(smem, w, Bm, C);
                const float sc = rw_cell_scale(lo, hi);
                rw_build(tab, A.bin_seed, bin_key(P, v, q0, p), B, lo, hi, sc);
                const RwBins bn{&tab, lo, sc};
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (lab[r] >= 0) atomicAdd(&hist[lab[r] * Bs + bn(val[r])], 1);
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (lab[r] >= 0) atomicAdd(&hist[lab[r] * Bs + bin_index(val[r], lo, scale, B)], 1);
            }
            wave_sync();
            LdsHistCM h{hist, Bs};
            write_hist_row(A, item_q(P, v, q0, p), h, B);
            float qm = -1.f;
            if (ENT) c = scan_hist_entropy(h, B, C, n, lo, scale, Flnk{block_flnk(smem, Bm, C, RW), kFlnkLds, nullptr, 0});
            else c = scan_hist_fast<!RW>(h, B, C, n, lo, scale, WS.pcs, bestq, &qm);
            if (RW && c.D != 0) c.thr = rw_boundary(A.bin_seed, bin_key(P, v, q0, p), B, lo, hi, c.pos);
            wave_sync();
            // a candidate is only returned valid when it may beat the incumbent
            if (c.D != 0 && cand_better(c, WS.best)) bestq = qm;
        }
        c.proj = p;
        const bool take = cand_better(c, WS.best);
        wave_sync();
        if (take && lane == 0) WS.best = c;
        wave_sync();
      }
    }
    __syncthreads();
    if (w == 0) {
        // the winning wave's index first, then one copy of its slot
        int bw = 0;
        for (int ww = 1; ww < kWavesPerBlock; ++ww)
            if (cand_better_proj(S.w[ww].best, S.w[bw].best)) bw = ww;
        Cand b = S.w[bw].best;
        uint64_t SP = 0;
        for (int c = 0; c < C; ++c) SP += (uint64_t)WS.pc[c] * (uint64_t)WS.pc[c];
        if (!ENT) b.SP = SP;
        if (lane == 0)
            write_record((SplitRec*)A.out + v, b, sortp ? SOF_SPLIT_SORT : (RW ? SOF_SPLIT_RHIST : SOF_SPLIT_HIST),
                         (int32_t)n, ENT);
    }
}

// item: (node, s0, n | k << 16, q0) as the plan wrote it
template <typename T, class PS, bool RW, bool ENT>
__device__ void do_small(const FindArgs& A, const PS& P, int4 it, char* smem) {
    const int v = it.x;
    const int64_t s0 = it.y;
    int64_t n = it.z & 0xffff;
    const int k = (int)((uint32_t)it.z >> 16), q0 = it.w;
    if (n > kSmallMax) n = kSmallMax;   // the plan never queues larger nodes here
    const int nr = (int)((n + kWave - 1) / kWave);
    if (nr <= 1) do_small_r<T, PS, 1, RW, ENT>(A, P, v, s0, n, k, q0, smem);
    else if (nr <= 2) do_small_r<T, PS, 2, RW, ENT>(A, P, v, s0, n, k, q0, smem);
    else if (nr <= 4) do_small_r<T, PS, 4, RW, ENT>(A, P, v, s0, n, k, q0, smem);
    else do_small_r<T, PS, kSmallR, RW, ENT>(A, P, v, s0, n, k, q0, smem);
}

// ---------------------------------------------------------------------------
// mid nodes: one block per (node, projection), 32 samples per thread

constexpr int kMidR = kMidMax / kBlock;   // up to 32 samples per thread

// A mid item carries everything its kernel needs to start: the node, its
// candidate slot base, the projection group, the node's projection count, its
// sample range and its first projection's index in the call (q0), so the
// kernel's first load is the item itself.
struct MidItem {
    int v, slot, g, k, s0, n, q0;
};

// Two-phase staging of a projection's nonzeros, so that a caller can overlap
// the CSR range loads with its own loads: stage_range reads the range of the
// projection with index q in the call (CSR; nothing for drawn projections),
// stage_fill stages the nonzeros into the wave's LDS (whole wave) and returns z.
struct StageRange {
    int64_t j0, j1;
};
__device__ __forceinline__ StageRange stage_range(const ProjCSR& P, int q) {
    q = q < P.n_proj ? (q < 0 ? 0 : q) : P.n_proj - 1;
    const int64_t j0 = clamp64(P.nz_offsets[q], 0, P.n_nz);
    int64_t j1 = clamp64(P.nz_offsets[q + 1], j0, P.n_nz);
    if (j1 - j0 > SOF_MAX_NNZ) j1 = j0 + SOF_MAX_NNZ;
    return StageRange{j0, j1};
}
__device__ __forceinline__ StageRange stage_range(const ProjHash&, int) { return StageRange{0, 0}; }
__device__ __forceinline__ int stage_fill(const ProjCSR& P, StageRange r, int, int, int d, int32_t* lf,
                                          uint32_t* ls) {
    const int z = (int)(r.j1 - r.j0);
    const int lane = lane_id();
    if (lane < z) {
        const uint32_t f = (uint32_t)P.nz_feature[r.j0 + lane];
        lf[lane] = f < (uint32_t)d ? (int)f : 0;
        ls[lane] = csr_weight_bits(P, r.j0 + lane);
    }
    wave_sync();
    return z;
}
__device__ __forceinline__ int stage_fill(const ProjHash& P, StageRange, int v, int p, int d, int32_t* lf,
                                          uint32_t* ls) {
    return proj_stage(P, v, p, d, lf, ls);
}

// One mid-node item: projections g*kMidGroup .. of node m.v, by one block.
// The node's row ids and labels are loaded once; wave j stages projection j's
// nonzeros; then for each projection all threads gather its values, the block
// reduces its range (one barrier) and counts it into that projection's own LDS
// histogram; finally wave j scans histogram j, so the group's scans run in
// parallel.  Range slots glo/ghi are indexed by projection, so no slot is
// rewritten while another wave may still read it.  The row ids and the CSR
// ranges are requested together, then the labels and the nonzeros, so the
// item costs two dependent round trips before its first gather.
template <typename T, class PS, int R, bool RW, bool ENT>
__device__ void do_mid_r(const FindArgs& A, const PS& P, const MidItem& m, int64_t n, char* smem) {
    BlockShared& S = block_shared(smem);
    const int tid = threadIdx.x, w = tid >> 6, lane = lane_id();
    const int C = A.n_classes, Bm = A.bins;
    const int v = m.v;
    const int64_t s0 = m.s0;
    const int B = node_bins(A, v);
    const int p0 = m.g * kMidGroup;
    const int np = m.k - p0 < kMidGroup ? m.k - p0 : kMidGroup;
    uint32_t rid[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = tid + (int64_t)r * kBlock;
        rid[r] = n > 0 ? (uint32_t)A.sample_idx[s0 + (i < n ? i : n - 1)] : 0u;
    }
    StageRange sr{0, 0};
    if (w < np) sr = stage_range(P, item_q(P, v, m.q0, p0 + w));
    uint32_t off[R];
    uint32_t labp[(R + 7) / 8];
#pragma unroll
    for (int q = 0; q < (R + 7) / 8; ++q) labp[q] = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = rid[r] < (uint32_t)A.n_rows ? (int)rid[r] : 0;
        off[r] = (uint32_t)row * (uint32_t)sizeof(T);
        labp[r >> 3] |= (uint32_t)label_of(A, row) << (4 * (r & 7));
    }
    if (w < np) {
        const int z = stage_fill(P, sr, v, p0 + w, A.n_features, S.w[w].lf, S.w[w].ls);
        if (lane == 0) S.gz[w] = z;
    }
    const int Bs = bins_stride(Bm);
    for (int j = 0; j < np; ++j) {
        int32_t* hist = wave_hist(smem, j, Bm, C);
        for (int e = tid * 4; e < C * Bs; e += kBlock * 4) *(int4*)(hist + e) = make_int4(0, 0, 0, 0);
    }
    __syncthreads();
    // Software pipeline over the group's projections: the first FB columns of
    // projection j + 1 are requested as soon as projection j's values are
    // complete, so their latency overlaps j's range barrier and histogram
    // (block barriers here wait for LDS only).  Adds stay in CSR order.
    constexpr int FB = R <= 8 ? 4 : (R <= 16 ? 2 : 1);
    float xa[FB][R];
    uint32_t sga[FB];
    int za = 0;
    auto request = [&](int j) {
        za = __builtin_amdgcn_readfirstlane(S.gz[j]);
        if (za > 0) {
#pragma unroll
            for (int t = 0; t < FB; ++t) {
                const int jt = t < za ? t : 0;
                const int f = __builtin_amdgcn_readfirstlane(S.w[j].lf[jt]);
                sga[t] = __builtin_amdgcn_readfirstlane(S.w[j].ls[jt]);
                const T* col = (const T*)A.x + (int64_t)f * A.ld;
#pragma unroll
                for (int r = 0; r < R; ++r) xa[t][r] = ldx_off(col, off[r]);
            }
        }
    };
    if (np > 0) request(0);
    for (int j = 0; j < np; ++j) {
        const int z = za;
        float val[R];
#pragma unroll
        for (int r = 0; r < R; ++r) val[r] = 0.f;
#pragma unroll
        for (int t = 0; t < FB; ++t) {
            if (t >= z) break;
#pragma unroll
            for (int r = 0; r < R; ++r) val[r] = __fadd_rn(val[r], weighted_term(xa[t][r], sga[t]));
        }
        for (int c = FB; c < z; ++c) {   // columns beyond the first FB, one round trip each
            const int f = __builtin_amdgcn_readfirstlane(S.w[j].lf[c]);
            const uint32_t sg = __builtin_amdgcn_readfirstlane(S.w[j].ls[c]);
            const T* col = (const T*)A.x + (int64_t)f * A.ld;
            float x[R];
#pragma unroll
            for (int r = 0; r < R; ++r) x[r] = ldx_off(col, off[r]);
#pragma unroll
            for (int r = 0; r < R; ++r) val[r] = __fadd_rn(val[r], weighted_term(x[r], sg));
        }
        if (j + 1 < np) request(j + 1);
        float lo = INFINITY, hi = -INFINITY;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (tid + (int64_t)r * kBlock < n) { lo = fminf(lo, val[r]); hi = fmaxf(hi, val[r]); }
        lo = wave_min_f(lo);
        hi = wave_max_f(hi);
        if (lane == 0) { S.glo[j][w] = lo; S.ghi[j][w] = hi; }
        __syncthreads();
        lo = fminf(fminf(S.glo[j][0], S.glo[j][1]), fminf(S.glo[j][2], S.glo[j][3]));
        hi = fmaxf(fmaxf(S.ghi[j][0], S.ghi[j][1]), fmaxf(S.ghi[j][2], S.ghi[j][3]));
        const float scale = bin_scale(B, lo, hi);
        int32_t* hist = wave_hist(smem, j, Bm, C);
        if (RW) {
            // every wave builds projection j's table in its own slot (no block barrier)
            RwTable& tab = wave_rw(smem, w, Bm, C);
            const float sc = rw_cell_scale(lo, hi);
            wave_sync();   // this wave's lookups of the previous projection are done
            rw_build(tab, A.bin_seed, bin_key(P, v, m.q0, p0 + j), B, lo, hi, sc);
            const RwBins bn{&tab, lo, sc};
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (tid + (int64_t)r * kBlock < n) {
                    const int y = (int)((labp[r >> 3] >> (4 * (r & 7))) & 15u);
                    atomicAdd(&hist[y * Bs + bn(val[r])], 1);
                }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (tid + (int64_t)r * kBlock < n) {
                    const int y = (int)((labp[r >> 3] >> (4 * (r & 7))) & 15u);
                    atomicAdd(&hist[y * Bs + bin_index(val[r], lo, scale, B)], 1);
                }
        }
    }
    __syncthreads();
    if (w < np) {
        const float lo = fminf(fminf(S.glo[w][0], S.glo[w][1]), fminf(S.glo[w][2], S.glo[w][3]));
        const float hi = fmaxf(fmaxf(S.ghi[w][0], S.ghi[w][1]), fmaxf(S.ghi[w][2], S.ghi[w][3]));
        const float scale = bin_scale(B, lo, hi);
        LdsHistCM h{wave_hist(smem, w, Bm, C), Bs};
        write_hist_row(A, item_q(P, v, m.q0, p0 + w), h, B);
        // the large instance (counts up to 8192, most above the LDS copy) reads the call's table only
        Cand c = ENT ? scan_hist_entropy(h, B, C, n, lo, scale,
                                         R <= 16 ? Flnk{block_flnk(smem, Bm, C, RW), kFlnkLds, A.ws.flnk, A.ws.cap_flnk}
                                                 : Flnk{nullptr, 0, A.ws.flnk, A.ws.cap_flnk})
                     : scan_hist_fast(h, B, C, n, lo, scale, S.w[w].pcs);
        if (RW && c.D != 0) c.thr = rw_boundary(A.bin_seed, bin_key(P, v, m.q0, p0 + w), B, lo, hi, c.pos);
        c.proj = p0 + w;
        if (lane == 0) ((Cand*)A.ws.slots)[m.slot + p0 + w] = c;
    }
}

// ---------------------------------------------------------------------------
// big nodes (more than 8192 samples, histogram path): the node's samples are
// cut into chunks of kChunk; a work item is one (projection, chunk) and is
// taken by one wave.  Items of big descriptor d are numbered
// item_a + p * nchunk + ch, and every per-item partial (range, histogram) is
// stored at that number.

// Item slots of a big node: k * nch, or in the XCD-local layout (nodes of
// kXcdChunks chunks or more) whole quads of projections times whole groups of
// kXcds chunks, plus room to start the region on a multiple of 4 * kXcds.
__host__ __device__ __forceinline__ bool big_xcd(int nch) { return nch >= kXcdChunks; }
__host__ __device__ __forceinline__ int big_slots(int k, int nch) {
    if (!big_xcd(nch)) return k * nch;
    return ((k + 3) / 4) * 4 * (((nch + kXcds - 1) / kXcds) * kXcds) + 4 * kXcds - 1;
}

struct BigDesc {
    int node, slot, item_a, item_c, bigslot, k, nchunk, vc;   // vc: value-cache base in kVcUnit units, or -1
};
__device__ __forceinline__ BigDesc big_desc(const FindArgs& A, int d) {
    int4 a = A.ws.desc_big[2 * d], b = A.ws.desc_big[2 * d + 1];
    return BigDesc{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
}

constexpr int kBR = 16;      // samples per lane per step of a range-pass chunk loop
constexpr int kBRHist = 8;   // ... of a histogram-pass chunk loop (fewer registers, more waves)

// Range (pass 1) or class histogram (pass 2) of projection p over chunk ch
// of a big node, by one wave.  Pass 2 counts into the wave's LDS histogram.
// Each step covers kWave * kR samples; the next step's row ids are loaded
// before this step's columns, and slots past the chunk's end repeat its last
// sample (valid addresses, masked out of the result).
template <typename T, class PS, bool kHist, class Bn>
__device__ __forceinline__ void big_chunk(const FindArgs& A, const PS& P, const BigDesc& bd, int p,
                                          int ch, WaveScratch& WS, float& lo, float& hi,
                                          int32_t* hist, const Bn& bin, float* vcw = nullptr) {
    constexpr int kR = kHist ? kBRHist : kBR;
    const int lane = lane_id();
    const int C = A.n_classes;
    int64_t s0, n;
    node_range(A, bd.node, s0, n);
    const int64_t c0 = (int64_t)ch * kChunk;
    const int cn = (int)clamp64(n - c0, 0, kChunk);
    const int z = __builtin_amdgcn_readfirstlane(proj_stage(P, bd.node, p, A.n_features, WS.lf, WS.ls));
    lo = INFINITY;
    hi = -INFINITY;
    if (cn <= 0) return;
    const int32_t* sidx = A.sample_idx + s0 + c0;
    int nxt[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int i = r * kWave + lane;
        nxt[r] = sidx[i < cn ? i : cn - 1];
    }
    for (int i0 = 0; i0 < cn; i0 += kWave * kR) {
        uint32_t off[kR];
        int lab[kR];
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const int row = (uint32_t)nxt[r] < (uint32_t)A.n_rows ? nxt[r] : 0;
            off[r] = (uint32_t)row * (uint32_t)sizeof(T);
            lab[r] = kHist ? label_of(A, row) : 0;
        }
        const int i1 = i0 + kWave * kR;
        if (i1 < cn) {
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const int i = i1 + r * kWave + lane;
                nxt[r] = sidx[i < cn ? i : cn - 1];
            }
        }
        float v[kR];
        gather_rows<T, kR>(A, WS.lf, WS.ls, z, off, v);
        if (!kHist && vcw) {
#pragma unroll
            for (int r = 0; r < kR; ++r)
                if (i0 + r * kWave + lane < cn) vcw[i0 + r * kWave + lane] = v[r];
        }
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            if (i0 + r * kWave + lane >= cn) continue;
            if (kHist) {
                atomicAdd(&hist[bin(v[r]) * C + lab[r]], 1);
            } else {
                lo = fminf(lo, v[r]);
                hi = fmaxf(hi, v[r]);
            }
        }
    }
}

// Histogram pass of (projection, chunk) from the value cache: the range pass
// stored the chunk's projected values, so only the row ids and labels are read
// besides them (coalesced, R per lane per step, slots past the end repeat the
// last sample and are masked out).
template <class Bn>
__device__ __forceinline__ void big_chunk_cached(const FindArgs& A, const BigDesc& bd, int ch, const float* vcr,
                                                 int32_t* hist, const Bn& bin) {
    const int lane = lane_id();
    const int C = A.n_classes;
    int64_t s0, n;
    node_range(A, bd.node, s0, n);
    const int64_t c0 = (int64_t)ch * kChunk;
    const int cn = (int)clamp64(n - c0, 0, kChunk);
    if (cn <= 0) return;
    const int32_t* sidx = A.sample_idx + s0 + c0;
    for (int i0 = 0; i0 < cn; i0 += kWave * kBRHist) {
        int lab[kBRHist];
        float v[kBRHist];
#pragma unroll
        for (int r = 0; r < kBRHist; ++r) {
            const int i = i0 + r * kWave + lane;
            const int j = i < cn ? i : cn - 1;
            const int row = (uint32_t)sidx[j] < (uint32_t)A.n_rows ? sidx[j] : 0;
            lab[r] = label_of(A, row);
            v[r] = vcr[j];
        }
#pragma unroll
        for (int r = 0; r < kBRHist; ++r)
            if (i0 + r * kWave + lane < cn) atomicAdd(&hist[bin(v[r]) * C + lab[r]], 1);
    }
}

// The value cache pays when re-gathering a projection costs more than
// reading its stored value back (z elements of s_x bytes against 4).
// vc >= 0: the cache's base; vc <= -2: base -2 - vc, and projections of at
// most 4 nonzeros re-gather (set by the expansion for XCD-local FP32 nodes
// whose distinct columns come to at most 8 bytes per value); -1: no cache.
__device__ __forceinline__ int vc_base(const BigDesc& bd) { return bd.vc >= 0 ? bd.vc : -2 - bd.vc; }
template <typename T>
__device__ __forceinline__ bool use_vcache(const BigDesc& bd, int z) {
    if (bd.vc == -1 || z * (int)sizeof(T) <= 8) return false;
    return bd.vc >= 0 || z > 4;
}
__device__ __forceinline__ float* vcache_at(const FindArgs& A, const BigDesc& bd, int p, int ch) {
    int64_t s0, n;
    node_range(A, bd.node, s0, n);
    return A.ws.vcache + (int64_t)vc_base(bd) * kVcUnit + (int64_t)p * n + (int64_t)ch * kChunk;
}

// ---------------------------------------------------------------------------
// kernels

__global__ void k_reset(int32_t* hdr) {
    for (int i = threadIdx.x; i < H_COUNT; i += blockDim.x) hdr[i] = 0;
}

template <class PS>
__global__ __launch_bounds__(kBlock) void k_plan(FindArgs A, PS P) {
    const int N = n_nodes_of(A);
    const FindWs& W = A.ws;
    for (int base = blockIdx.x * kBlock; base < N; base += gridDim.x * kBlock) {
        const int v = base + threadIdx.x;
        const bool act = v < N;
        int64_t s0 = 0, n = 0;
        int k = 0;
        if (act) {
            node_range(A, v, s0, n);
            k = proj_count(P, v);
        }
        const bool sortp = n < A.sort_threshold;
        int cat = CAT_NONE;
        if (act) {
            if (k == 0) cat = CAT_NOSPLIT;
            else if (sortp ? n <= kSortWaveMax : n <= A.small_max) cat = CAT_SMALL;
            else if (sortp) cat = CAT_SB;
            else if (n <= A.mid_split) cat = CAT_MID;
            else if (n <= kMidMax) cat = CAT_MID2;
            else cat = CAT_BIG;
        }
        const int nch = (int)((n + kChunk - 1) / kChunk);
        const bool slot_node = cat == CAT_MID || cat == CAT_MID2 || cat == CAT_SB || cat == CAT_BIG;
        const int gmid = (k + kMidGroup - 1) / kMidGroup;
        const int vunits = cat == CAT_BIG ? (int)((n * (int64_t)k + kVcUnit - 1) / kVcUnit) : 0;
        const int ctr[13] = {H_SMALL, H_DMID, H_IMID, H_DMID2, H_IMID2, H_DSB, H_ISB,
                             H_DBIG, H_IBIGA, H_IBIGC, H_SLOTS, H_BIGSLOTS, H_VCACHE};
        const int cnt[13] = {cat == CAT_SMALL, cat == CAT_MID, cat == CAT_MID ? gmid : 0,
                             cat == CAT_MID2, cat == CAT_MID2 ? gmid : 0, cat == CAT_SB, cat == CAT_SB ? k : 0,
                             cat == CAT_BIG, cat == CAT_BIG ? big_slots(k, nch) : 0, cat == CAT_BIG ? k : 0,
                             slot_node ? k : 0, cat == CAT_BIG ? k : 0, vunits};
        int ob[13];
        wave_alloc_n<13>(W.hdr, ctr, cnt, ob);
        const int o_small = ob[0], o_dmid = ob[1], o_imid = ob[2], o_dmid2 = ob[3], o_imid2 = ob[4];
        const int o_dsb = ob[5], o_isb = ob[6], o_dbig = ob[7], o_ia = ob[8], o_ic = ob[9];
        const int o_slot = ob[10], o_bslot = ob[11], o_vc = ob[12];
        bool over = false;
        if (slot_node && o_slot + (int64_t)k > W.cap_slots) over = true;
        if (cat == CAT_SMALL && o_small >= W.cap_small) over = true;
        if (cat == CAT_MID && (o_dmid >= W.cap_dmid || o_imid + (int64_t)gmid > W.cap_imid)) over = true;
        if (cat == CAT_MID2 && (o_dmid2 >= W.cap_dmid2 || o_imid2 + (int64_t)gmid > W.cap_imid2)) over = true;
        if (cat == CAT_SB && (o_dsb >= W.cap_dsb || o_isb + (int64_t)k > W.cap_isb)) over = true;
        if (cat == CAT_BIG && (o_dbig >= W.cap_dbig || o_ia + (int64_t)big_slots(k, nch) > W.cap_ibiga ||
                               o_ic + (int64_t)k > W.cap_ibigc || o_bslot + (int64_t)k > W.cap_bigslots))
            over = true;
        if (over) {
            // Capacity exceeded (impossible with truthful host-side sizes): flag
            // it, record no split, and leave an empty descriptor so that every
            // allocated descriptor slot below the capacity is initialised.
            atomicOr(&W.hdr[H_ERR], 1);
            write_nosplit(A, v, sortp ? 1 : 0, n);
            if (cat == CAT_MID && o_dmid < W.cap_dmid) W.desc_mid[o_dmid] = make_int4(v, 0, 0, 0);
            if (cat == CAT_MID2 && o_dmid2 < W.cap_dmid2) W.desc_mid2[o_dmid2] = make_int4(v, 0, 0, 0);
            if (cat == CAT_SB && o_dsb < W.cap_dsb) W.desc_sb[o_dsb] = make_int4(v, 0, 0, 0);
            if (cat == CAT_BIG && o_dbig < W.cap_dbig) {
                W.desc_big[2 * o_dbig] = make_int4(v, 0, 0, 0);
                W.desc_big[2 * o_dbig + 1] = make_int4(0, 0, 0, 0);
            }
            continue;
        }
        switch (cat) {
        case CAT_NOSPLIT: write_nosplit(A, v, sortp ? 1 : 0, n); break;
        case CAT_SMALL:
            // k <= max_proj_per_node <= 1024 by contract; clamped so the pack stays defined
            W.small_items[o_small] =
                make_int4(v, (int)s0, (int)((uint32_t)n | ((uint32_t)(k < 0x7fff ? k : 0x7fff) << 16)),
                          proj_global(P, v, 0));
            break;
        case CAT_MID: W.desc_mid[o_dmid] = make_int4(v, o_slot, o_imid, k); break;
        case CAT_MID2: W.desc_mid2[o_dmid2] = make_int4(v, o_slot, o_imid2, k); break;
        case CAT_SB: W.desc_sb[o_dsb] = make_int4(v, o_slot, o_isb, k); break;
        case CAT_BIG:
            W.desc_big[2 * o_dbig] = make_int4(v, o_slot, o_ia, o_ic);
            W.desc_big[2 * o_dbig + 1] =
                make_int4(o_bslot, k, nch, o_vc >= 0 && o_vc + (int64_t)vunits <= W.cap_vcache ? o_vc : -1);
            break;
        default: break;
        }
    }
}

constexpr int kMaxProj = 1024;   // projections per node (the boundary's limit)
constexpr int kExpandSlices = 16;   // blocks sharing the item writes of one big node

template <class PS>
__global__ __launch_bounds__(kBlock) void k_expand(FindArgs A, PS P) {
    __shared__ int zcnt[SOF_MAX_NNZ + 1], zbase[SOF_MAX_NNZ + 1];
    __shared__ int perm[kMaxProj];
    __shared__ uint8_t zof[kMaxProj];
    const FindWs& W = A.ws;
    const int tid = threadIdx.x;
    const int nmid = count_of(A, H_DMID, W.cap_dmid);
    const int nsb = count_of(A, H_DSB, W.cap_dsb);
    const int nbig = count_of(A, H_DBIG, W.cap_dbig);
    const int nmid2 = count_of(A, H_DMID2, W.cap_dmid2);
    // a big descriptor is written by kExpandSlices blocks, each a slice of its items
    for (int d = blockIdx.x; d < nmid + nsb + nbig * kExpandSlices + nmid2; d += gridDim.x) {
        if (d >= nmid + nsb + nbig * kExpandSlices) {
            const int e = d - nmid - nsb - nbig * kExpandSlices;
            const int4 D = W.desc_mid2[e];
            const int ng = (D.w + kMidGroup - 1) / kMidGroup;
            int64_t s0 = 0, n = 0;
            if (ng > 0) node_range(A, D.x, s0, n);
            const int q0 = ng > 0 ? proj_global(P, D.x, 0) : 0;
            for (int g = tid; g < ng; g += kBlock)
                if (D.z + (int64_t)g < W.cap_imid2) {
                    W.items_mid2[2 * (D.z + g)] = make_int4(D.x, D.y, g, D.w);
                    W.items_mid2[2 * (D.z + g) + 1] = make_int4((int)s0, (int)n, q0, 0);
                }
        } else if (d < nmid) {
            const int4 D = W.desc_mid[d];
            const int ng = (D.w + kMidGroup - 1) / kMidGroup;
            int64_t s0 = 0, n = 0;
            if (ng > 0) node_range(A, D.x, s0, n);
            const int q0 = ng > 0 ? proj_global(P, D.x, 0) : 0;
            for (int g = tid; g < ng; g += kBlock)
                if (D.z + (int64_t)g < W.cap_imid) {
                    W.items_mid[2 * (D.z + g)] = make_int4(D.x, D.y, g, D.w);
                    W.items_mid[2 * (D.z + g) + 1] = make_int4((int)s0, (int)n, q0, 0);
                }
        } else if (d < nmid + nsb) {
            int e = d - nmid;
            int4 D = W.desc_sb[e];
            for (int p = tid; p < D.w; p += kBlock)
                if (D.z + (int64_t)p < W.cap_isb) W.items_sb[D.z + p] = make_int2(e, p);
        } else {
            // (projection, chunk) items with the projections ordered by
            // nonzero count, most first: a round of grid-stride items then
            // holds items of about equal cost, so the statically assigned
            // rounds of the big-node kernels stay balanced when the counts
            // vary.  Item t of the node stands for (p, ch) with
            // t' = p * nchunk + ch (stored), wherever it sits; the range and
            // histogram results are indexed by t' and merged order-free, so
            // the order changes no result.
            const int e = (d - nmid - nsb) / kExpandSlices, slice = (d - nmid - nsb) % kExpandSlices;
            BigDesc bd = big_desc(A, e);
            const int k = bd.k < kMaxProj ? bd.k : kMaxProj;
            const int na = big_slots(bd.k, bd.nchunk);
            const int t0 = (int)((int64_t)na * slice / kExpandSlices);
            const int t1 = (int)((int64_t)na * (slice + 1) / kExpandSlices);
            // The order is a function of the counts alone (equal counts by
            // projection index), so every slice block builds the same one.
            if (tid <= SOF_MAX_NNZ) zcnt[tid] = 0;
            __syncthreads();
            int zr[kMaxProj / kBlock];
#pragma unroll
            for (int i = 0; i < kMaxProj / kBlock; ++i) {
                const int p = tid + i * kBlock;
                zr[i] = p < k ? proj_nnz(P, bd.node, p, A.n_features) : 0;
                if (p < k) {
                    zof[p] = (uint8_t)zr[i];
                    atomicAdd(&zcnt[zr[i]], 1);
                }
            }
            __syncthreads();
            if (tid == 0) {
                int b = 0;
                for (int z = SOF_MAX_NNZ; z >= 0; --z) { zbase[z] = b; b += zcnt[z]; }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < kMaxProj / kBlock; ++i) {
                const int p = tid + i * kBlock;
                if (p < k) {
                    int before = 0;   // projections below p with the same count
                    for (int q = 0; q < p; ++q) before += zof[q] == zr[i] ? 1 : 0;
                    perm[zbase[zr[i]] + before] = p;
                }
            }
            __syncthreads();
            if (!big_xcd(bd.nchunk)) {
                for (int t = t0 + tid; t < t1; t += kBlock) {
                    const int pos = t / bd.nchunk, ch = t - pos * bd.nchunk;
                    if (bd.item_a + (int64_t)t < W.cap_ibiga)
                        W.items_biga[bd.item_a + t] = make_int2(e, perm[pos] * bd.nchunk + ch);
                }
            } else {
                // XCD-local layout: in the static rounds slot s of the items
                // array goes to a wave of block s / 4 (mod the grid, a multiple
                // of kXcds blocks), which runs on XCD (s / 4) mod kXcds.  The
                // region starts on a multiple of 4 kXcds, and its slot
                // a = 4 kXcds q + 4 x + j holds chunk kXcds g + x and projection
                // position 4 pq + j, q = g Q4 + pq: every projection of a chunk
                // runs on one XCD at about the same time, so the chunk's columns
                // are read from HBM about once and then from that XCD's L2.
                // Slots past the node's chunks or projections hold no item.
                const int Q4 = (bd.k + 3) / 4;
                const int nreg = Q4 * 4 * (((bd.nchunk + kXcds - 1) / kXcds) * kXcds);
                const int base = ((bd.item_a + 4 * kXcds - 1) & ~(4 * kXcds - 1)) - bd.item_a;
                for (int t = t0 + tid; t < t1; t += kBlock) {
                    int2 item = make_int2(-1, 0);
                    const int a = t - base;
                    if (a >= 0 && a < nreg) {
                        const int q = a / (4 * kXcds), x = (a >> 2) % kXcds, j = a & 3;
                        const int g = q / Q4, pq = q - g * Q4;
                        const int ch = g * kXcds + x, pos = pq * 4 + j;
                        if (ch < bd.nchunk && pos < k) item = make_int2(e, perm[pos] * bd.nchunk + ch);
                    }
                    if (bd.item_a + (int64_t)t < W.cap_ibiga) W.items_biga[bd.item_a + t] = item;
                }
            }
            if (slice == 0) {
                for (int p = tid; p < bd.k; p += kBlock)
                    if (bd.item_c + (int64_t)p < W.cap_ibigc) W.items_bigc[bd.item_c + p] = make_int2(e, p);
                // In the XCD-local layout, FP32 projections of at most 4
                // nonzeros whose node reads at most 8 bytes of distinct
                // columns per value (min(d, sum z) columns over k projections)
                // re-gather from L2 in the histogram pass instead of writing
                // and reading the value cache (8 bytes of HBM per value).
                // Projections of more nonzeros, and FP16 gathers (128 bytes
                // per wave instruction), are bound by their issue and keep it.
                int zs = 0;
                for (int z = 1; z <= SOF_MAX_NNZ; ++z) zs += z * zcnt[z];
                const int64_t m = zs < A.n_features ? zs : A.n_features;
                if (tid == 0 && bd.vc >= 0 && big_xcd(bd.nchunk) && A.dtype != SOF_F16 &&
                    m * 4 <= 8 * (int64_t)bd.k)
                    ((int*)&W.desc_big[2 * e + 1])[3] = -2 - bd.vc;
            }
            __syncthreads();   // zcnt and perm are reused by the block's next descriptor
        }
    }
}

// Per-wave items 0 .. n-1.  All but the last kDynRounds rounds of grid-stride
// items are taken statically (no atomics, no barriers); the rest are claimed
// dynamically, kWavesPerBlock consecutive items per block claim (one atomic,
// wave w takes the w-th), so waves whose items cost more (more nonzeros) or
// that became resident late (the size classes share the GPU) take fewer of
// the tail; with at most kStaticRounds rounds every item is taken statically.
// body(it) runs on whole waves and contains no block barrier.
constexpr int kDynRounds = 1;
constexpr int kStaticRounds = 2;   // up to this many rounds: static grid stride only
template <class F>
__device__ __forceinline__ void for_wave_items(int n, int32_t* ctr, int* s_item, F&& body) {
    const int w = threadIdx.x >> 6;
    const int gw = (int)((blockIdx.x * kBlock + threadIdx.x) >> 6);
    const int nw = (int)(gridDim.x * kWavesPerBlock);
    if (n <= kStaticRounds * nw) {   // few rounds (cheap, even items): no claims at all
        for (int it = gw; it < n; it += nw) body(it);
        return;
    }
    const int fixed = n / nw - kDynRounds;
    for (int r = 0; r < fixed; ++r) body(gw + r * nw);
    const int base = (fixed > 0 ? fixed : 0) * nw;
    for (;;) {
        const int first = base + block_dequeue(ctr, s_item) * kWavesPerBlock;
        if (first >= n) break;
        if (first + w < n) body(first + w);
    }
}

// big item it -> (descriptor, projection, chunk); false if out of range
__device__ __forceinline__ bool big_item(const FindArgs& A, int it, int nbig, BigDesc& bd, int& p,
                                         int& ch) {
    const int2 e = A.ws.items_biga[it];
    if (e.x < 0 || e.x >= nbig) return false;
    bd = big_desc(A, e.x);
    if (bd.nchunk <= 0 || e.y < 0 || e.y >= bd.k * bd.nchunk) return false;
    p = e.y / bd.nchunk;
    ch = e.y - p * bd.nchunk;
    return true;
}

template <typename T, class PS>
__global__ __launch_bounds__(kBlock) void k_brange(FindArgs A, PS P) {
    extern __shared__ __align__(16) char smem[];
    BlockShared& S = block_shared(smem);
    const FindWs& W = A.ws;
    const int na = count_of(A, H_IBIGA, W.cap_ibiga);
    const int nbig = count_of(A, H_DBIG, W.cap_dbig);
    WaveScratch& WS = S.w[threadIdx.x >> 6];
    for_wave_items(na, &W.hdr[H_Q_BRANGE], &S.item, [&](int it) {
        BigDesc bd;
        int p, ch;
        if (!big_item(A, it, nbig, bd, p, ch)) return;
        float lo, hi;
        float* vcw = use_vcache<T>(bd, proj_nnz(P, bd.node, p, A.n_features)) ? vcache_at(A, bd, p, ch) : nullptr;
        big_chunk<T, PS, false>(A, P, bd, p, ch, WS, lo, hi, nullptr, EqualBins{0.f, 0.f, 2}, vcw);
        lo = wave_min(lo);
        hi = wave_max(hi);
        if (lane_id() == 0) W.crange[bd.item_a + (int64_t)p * bd.nchunk + ch] = make_float2(lo, hi);
    });
}

// range of every (big node, projection): min and max over its chunks
__global__ __launch_bounds__(kBlock) void k_bmerge(FindArgs A) {
    __shared__ int s_item;
    const FindWs& W = A.ws;
    const int nc = count_of(A, H_IBIGC, W.cap_ibigc);
    const int nbig = count_of(A, H_DBIG, W.cap_dbig);
    for_wave_items(nc, &W.hdr[H_Q_BMERGE], &s_item, [&](int it) {
        const int2 e = W.items_bigc[it];
        if (e.x < 0 || e.x >= nbig) return;
        const BigDesc bd = big_desc(A, e.x);
        const int p = e.y;
        if (p < 0 || p >= bd.k) return;
        float lo = INFINITY, hi = -INFINITY;
        const int64_t base = (int64_t)bd.item_a + (int64_t)p * bd.nchunk;
        for (int ch = lane_id(); ch < bd.nchunk; ch += kWave) {
            if (base + ch >= W.cap_ibiga) break;
            const float2 r = W.crange[base + ch];
            lo = fminf(lo, r.x);
            hi = fmaxf(hi, r.y);
        }
        lo = wave_min(lo);
        hi = wave_max(hi);
        if (bd.bigslot + (int64_t)p < W.cap_bigslots) {
            if (lane_id() == 0) W.brange[bd.bigslot + p] = make_float2(lo, hi);
            // the projection's histogram, filled by the histogram pass
            int32_t* ph = W.phist + (int64_t)(bd.bigslot + p) * A.bins * A.n_classes;
            for (int e = lane_id(); e < A.bins * A.n_classes; e += kWave) ph[e] = 0;
        }
    });
}

template <typename T, class PS, bool RW>
__global__ __launch_bounds__(kBlock) void k_bhist(FindArgs A, PS P) {
    extern __shared__ __align__(16) char smem[];
    BlockShared& S = block_shared(smem);
    const FindWs& W = A.ws;
    const int na = count_of(A, H_IBIGA, W.cap_ibiga);
    const int nbig = count_of(A, H_DBIG, W.cap_dbig);
    const int w = threadIdx.x >> 6, lane = lane_id();
    const int C = A.n_classes, Bm = A.bins;
    WaveScratch& WS = S.w[w];
    int32_t* hist = wave_hist(smem, w, Bm, C);
    for_wave_items(na, &W.hdr[H_Q_BHIST], &S.item, [&](int it) {
        BigDesc bd;
        int p, ch;
        if (!big_item(A, it, nbig, bd, p, ch)) return;
        if (bd.bigslot + (int64_t)p >= W.cap_bigslots) return;
        const int B = node_bins(A, bd.node);
        const float2 r = W.brange[bd.bigslot + p];
        const float scale = bin_scale(B, r.x, r.y);
        for (int e = lane; e < B * C; e += kWave) hist[e] = 0;
        wave_sync();
        float lo, hi;
        const float* vcr = use_vcache<T>(bd, proj_nnz(P, bd.node, p, A.n_features)) ? vcache_at(A, bd, p, ch) : nullptr;
        if (RW) {
            RwTable& tab = wave_rw(smem, w, Bm, C);
            const float sc = rw_cell_scale(r.x, r.y);
            rw_build(tab, A.bin_seed, bin_key(P, bd.node, proj_global(P, bd.node, 0), p), B, r.x, r.y, sc);
            if (vcr) big_chunk_cached(A, bd, ch, vcr, hist, RwBins{&tab, r.x, sc});
            else big_chunk<T, PS, true>(A, P, bd, p, ch, WS, lo, hi, hist, RwBins{&tab, r.x, sc});
        } else {
            if (vcr) big_chunk_cached(A, bd, ch, vcr, hist, EqualBins{r.x, scale, B});
            else big_chunk<T, PS, true>(A, P, bd, p, ch, WS, lo, hi, hist, EqualBins{r.x, scale, B});
        }
        wave_sync();
        // add the chunk's counts into the projection's histogram (integer
        // additions commute, so the sum does not depend on their order)
        int32_t* ph = W.phist + (int64_t)(bd.bigslot + p) * Bm * C;
        for (int e = lane; e < B * C; e += kWave)
            if (hist[e]) atomicAdd(&ph[e], hist[e]);
        wave_sync();
    });
}

// Per (big node, projection): the projection's histogram (summed by the
// histogram pass) into the wave's LDS histogram, then the boundary scan.
template <class PS, bool RW, bool ENT>
__global__ __launch_bounds__(kBlock) void k_bscan(FindArgs A, PS P) {
    extern __shared__ __align__(16) char smem[];
    const FindWs& W = A.ws;
    const int nc = count_of(A, H_IBIGC, W.cap_ibigc);
    const int nbig = count_of(A, H_DBIG, W.cap_dbig);
    const int w = threadIdx.x >> 6, lane = lane_id();
    const int C = A.n_classes, Bm = A.bins;
    int32_t* hist = wave_hist(smem, w, Bm, C);
    for_wave_items(nc, &W.hdr[H_Q_BSCAN], &block_shared(smem).item, [&](int it) {
        const int2 e = W.items_bigc[it];
        if (e.x < 0 || e.x >= nbig) return;
        const BigDesc bd = big_desc(A, e.x);
        const int p = e.y;
        if (p < 0 || p >= bd.k || bd.bigslot + (int64_t)p >= W.cap_bigslots ||
            bd.slot + (int64_t)p >= W.cap_slots)
            return;
        const int B = node_bins(A, bd.node);
        int64_t s0, n;
        node_range(A, bd.node, s0, n);
        const int Bs = bins_stride(Bm);
        const int32_t* ph = W.phist + (int64_t)(bd.bigslot + p) * Bm * C;
        for (int e = lane; e < C * Bs; e += kWave) {
            const int c = e / Bs, b = e - c * Bs;
            hist[e] = b < B ? ph[b * C + c] : 0;
        }
        wave_sync();
        const float2 r = W.brange[bd.bigslot + p];
        const float scale = bin_scale(B, r.x, r.y);
        LdsHistCM h{hist, Bs};
        write_hist_row(A, proj_global(P, bd.node, p), h, B);
        Cand c = ENT ? scan_hist_entropy(h, B, C, n, r.x, scale, Flnk{nullptr, 0, A.ws.flnk, A.ws.cap_flnk})
                     : scan_hist_fast(h, B, C, n, r.x, scale, block_shared(smem).w[w].pcs);
        if (RW && c.D != 0) c.thr = rw_boundary(A.bin_seed, bin_key(P, bd.node, proj_global(P, bd.node, 0), p), B, r.x, r.y, c.pos);
        c.proj = p;
        if (lane == 0) ((Cand*)W.slots)[bd.slot + p] = c;
        wave_sync();
    });
}

// kLarge: nodes of kMidSplit+1 .. kMidMax samples (32 per thread); else
// kSmallMax+1 .. kMidSplit (up to 16 per thread).  Separate kernels so that
// each gets the register allocation of its own size class.
template <typename T, class PS, bool kLarge, bool RW, bool ENT>
__global__ __launch_bounds__(kBlock, kLarge ? 1 : 4) void k_mid(FindArgs A, PS P) {
    extern __shared__ __align__(16) char smem[];
    BlockShared& S = block_shared(smem);
    const FindWs& W = A.ws;
    const int nm = kLarge ? count_of(A, H_IMID2, W.cap_imid2) : count_of(A, H_IMID, W.cap_imid);
    const int4* items = kLarge ? W.items_mid2 : W.items_mid;
    const int N = n_nodes_of(A);
    if (ENT && !kLarge) fill_flnk<RW>(A, smem);   // the first dequeue's barrier publishes it
    for (;;) {
        int it = block_dequeue(&W.hdr[kLarge ? H_Q_MID2 : H_Q_MID], &S.item);
        if (it >= nm) break;
        const int4 a = items[2 * it], b = items[2 * it + 1];
        const MidItem m{a.x, a.y, a.z, a.w, b.x, b.y, b.z};
        if (m.v < 0 || m.v >= N || m.g < 0 || m.g * kMidGroup >= m.k || m.s0 < 0 || m.n < 0 ||
            (int64_t)m.s0 + m.n > A.n_samples || m.slot < 0 || (int64_t)m.slot + m.k > W.cap_slots)
            continue;
        int64_t n = m.n;
        if (kLarge) {
            if (n > kMidMax) n = kMidMax;   // the plan never queues larger nodes here
            do_mid_r<T, PS, kMidR, RW, ENT>(A, P, m, n, smem);
        } else {
            if (n > kMidSplit) n = kMidSplit;   // the plan never queues larger nodes here
            const int nr = (int)((n + kBlock - 1) / kBlock);
            if (nr <= 4) do_mid_r<T, PS, 4, RW, ENT>(A, P, m, n, smem);
            else if (nr <= 8) do_mid_r<T, PS, 8, RW, ENT>(A, P, m, n, smem);
            else do_mid_r<T, PS, 16, RW, ENT>(A, P, m, n, smem);
        }
    }
}

template <typename T, class PS, bool RW, bool ENT>
__global__ __launch_bounds__(kBlock, 4) void k_small(FindArgs A, PS P) {
    extern __shared__ __align__(16) char smem[];
    BlockShared& S = block_shared(smem);
    const FindWs& W = A.ws;
    const int ns = count_of(A, H_SMALL, W.cap_small);
    const int N = n_nodes_of(A);
    if (ENT) fill_flnk<RW>(A, smem);   // the first dequeue's barrier publishes it
    for (;;) {
        int it = block_dequeue(&W.hdr[H_Q_SMALL], &S.item);
        if (it >= ns) break;
        const int4 e = W.small_items[it];
        const int64_t n = e.z & 0xffff;
        if (e.x >= 0 && e.x < N && e.y >= 0 && (int64_t)e.y + n <= A.n_samples)
            do_small<T, PS, RW, ENT>(A, P, e, smem);
    }
}

__global__ __launch_bounds__(kBlock) void k_reduce(FindArgs A) {
    const FindWs& W = A.ws;
    const int nmid = count_of(A, H_DMID, W.cap_dmid);
    const int nsb = count_of(A, H_DSB, W.cap_dsb);
    const int nbig = count_of(A, H_DBIG, W.cap_dbig);
    const int nmid2 = count_of(A, H_DMID2, W.cap_dmid2);
    const int lane = lane_id();
    const Cand* slots = (const Cand*)W.slots;
    const int gw = (blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int nw = gridDim.x * kWavesPerBlock;
    const int hist_kind = A.bin_mode == SOF_BINS_RANDOM ? SOF_SPLIT_RHIST : SOF_SPLIT_HIST;
    for (int d = gw; d < nmid + nsb + nbig + nmid2; d += nw) {
        int node, slot, k, kind;
        if (d >= nmid + nsb + nbig) {
            int4 D = W.desc_mid2[d - nmid - nsb - nbig]; node = D.x; slot = D.y; k = D.w; kind = hist_kind;
        } else if (d < nmid) {
            int4 D = W.desc_mid[d]; node = D.x; slot = D.y; k = D.w; kind = hist_kind;
        } else if (d < nmid + nsb) {
            int4 D = W.desc_sb[d - nmid]; node = D.x; slot = D.y; k = D.w; kind = 1;
        } else {
            BigDesc bd = big_desc(A, d - nmid - nsb); node = bd.node; slot = bd.slot; k = bd.k; kind = hist_kind;
        }
        if (slot + (int64_t)k > W.cap_slots) continue;
        bool bv = false;
        u128 bN = 0;
        uint64_t bD = 0;
        int bp = 0;
        for (int p = lane; p < k; p += kWave) {
            const Cand& c = slots[slot + p];
            if (c.D != 0 && (!bv || q_greater(c.N, c.D, bN, bD))) { bv = true; bN = c.N; bD = c.D; bp = p; }
        }
        int win = wave_best_lane(bv, bN, bD, bp);
        int64_t s0, n;
        node_range(A, node, s0, n);
        Cand b;
        if (win >= 0) b = slots[slot + __shfl(bp, win)];
        else cand_invalid(b);
        if (lane == 0) write_record((SplitRec*)A.out + node, b, kind, (int32_t)n, A.criterion == SOF_CRIT_ENTROPY);
    }
}

// ---------------------------------------------------------------------------
// sort-path blocks: 64 < n <= 8192, bitonic sort of (key, label) in LDS

struct SortShared {
    int item;
    int z;
    int pad[2];
    int32_t lf[16];
    uint32_t ls[16];
    int32_t pc[16];
    uint64_t wtot[kWavesPerBlock][4];
    uint64_t wN[kWavesPerBlock][2];
    uint64_t wD[kWavesPerBlock];
    uint64_t wSL[kWavesPerBlock];
    uint64_t wSR[kWavesPerBlock];
    int32_t wpos[kWavesPerBlock];
};

size_t find_smem_sort() { return sizeof(SortShared) + (size_t)kSortMax * sizeof(uint64_t); }

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t x) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        uint64_t t = __shfl_up(x, off);
        if (lane >= off) x += t;
    }
    return x;
}

// One (node, projection) of a sort-path node with 64 < n <= 8192: project
// into LDS as (order-preserving key << 32 | label), bitonic sort, then each
// thread scans a contiguous run of sorted positions with 16-bit packed class
// counters (four classes per 64-bit word) offset by a block prefix sum.
// ENT: the entropy criterion (as in scan_sort_small), f(k) from the call's
// table.
template <typename T, class PS, bool ENT>
__device__ void do_sortblock(const FindArgs& A, const PS& P, int4 D, int p, char* smem) {
    SortShared& S = *(SortShared*)smem;
    uint64_t* keys = (uint64_t*)(smem + sizeof(SortShared));
    const int tid = threadIdx.x, w = tid >> 6, lane = lane_id();
    const int C = A.n_classes;
    const int v = D.x;
    int64_t s0, n;
    node_range(A, v, s0, n);
    if (n > kSortMax) n = kSortMax;   // cannot happen: the threshold is clamped on the host
    int P2 = 128;
    while (P2 < n) P2 <<= 1;
    if (w == 0) {
        int z = proj_stage(P, v, p, A.n_features, S.lf, S.ls);
        if (lane == 0) S.z = z;
        if (lane < 16) S.pc[lane] = 0;
    }
    __syncthreads();
    const int zn = S.z;
    for (int i = tid; i < P2; i += kBlock) {
        uint64_t key = ~0ull;
        if (i < n) {
            const int row = row_of(A, s0 + i);
            const int y = label_of(A, row);
            float acc = 0.f;
            for (int j = 0; j < zn; ++j) {
                const T* col = (const T*)A.x + (int64_t)S.lf[j] * A.ld;
                acc = __fadd_rn(acc, weighted_term(ldx(col, row), S.ls[j]));
            }
            atomicAdd(&S.pc[y], 1);
            key = ((uint64_t)fkey(acc) << 32) | (uint32_t)y;
        }
        keys[i] = key;
    }
    __syncthreads();
    for (int kk = 2; kk <= P2; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            const int lj = __ffs(j) - 1;
            for (int t = tid; t < (P2 >> 1); t += kBlock) {
                const int i = ((t >> lj) << (lj + 1)) + (t & (j - 1));
                const int l = i + j;
                const bool asc = (i & kk) == 0;
                const uint64_t a = keys[i], b = keys[l];
                if ((a > b) == asc) { keys[i] = b; keys[l] = a; }
            }
            __syncthreads();
        }
    }
    const int E = P2 >= kBlock ? P2 / kBlock : 1;
    const int t0 = tid * E;
    const int CW = (C + 3) >> 2;
    uint64_t loc[4] = {0, 0, 0, 0};
    for (int e = 0; e < E; ++e) {
        const int i = t0 + e;
        if (i < n) {
            const int y = (int)(uint32_t)keys[i];
            const uint64_t one = 1ull << (16 * (y & 3));
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (q == (y >> 2)) loc[q] += one;
        }
    }
    uint64_t excl[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint64_t incl = q < CW ? wave_incl_scan64(loc[q]) : 0ull;
        excl[q] = incl - loc[q];
        if (lane == 63) S.wtot[w][q] = incl;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q)
        for (int ww = 0; ww < w; ++ww) excl[q] += S.wtot[ww][q];
    const Flnk tab{nullptr, 0, A.ws.flnk, A.ws.cap_flnk};
    uint64_t SP = 0;
    if (ENT) {
        double FP = 0.0;
        for (int c = 0; c < C; ++c) FP = __dadd_rn(FP, flnk_at(tab, S.pc[c]));
        SP = d_bits(FP);
    } else {
        for (int c = 0; c < C; ++c) SP += (uint64_t)S.pc[c] * (uint64_t)S.pc[c];
    }
    bool bv = false;
    u128 bN = 0;
    uint64_t bD = 0, bSL = 0, bSR = 0;
    int bpos = 0;
    uint64_t cur[4] = {excl[0], excl[1], excl[2], excl[3]};
    for (int e = 0; e < E; ++e) {
        const int i = t0 + e;
        if (i >= n) break;
        const uint64_t ki = keys[i];
        const int y = (int)(uint32_t)ki;
        const uint64_t one = 1ull << (16 * (y & 3));
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q == (y >> 2)) cur[q] += one;
        if (ENT && i + 1 < n && (uint32_t)(ki >> 32) < (uint32_t)(keys[i + 1] >> 32)) {
            double FL = 0.0, FR = 0.0;
            for (int c = 0; c < C; ++c) {
                const uint32_t l = (uint32_t)((cur[c >> 2] >> (16 * (c & 3))) & 0xffffu);
                FL = __dadd_rn(FL, flnk_at(tab, l));
                FR = __dadd_rn(FR, flnk_at(tab, (uint32_t)S.pc[c] - l));
            }
            const double Ev = __dsub_rn(__dsub_rn(__dadd_rn(FL, FR), flnk_at(tab, (int64_t)i + 1)),
                                        flnk_at(tab, n - i - 1));
            const u128 N = (u128)dkey(Ev);
            if (!bv || N > bN) { bv = true; bN = N; bD = 1; bpos = i; bSL = d_bits(FL); bSR = d_bits(FR); }
        } else if (!ENT && i + 1 < n && (uint32_t)(ki >> 32) < (uint32_t)(keys[i + 1] >> 32)) {
            uint64_t SL = 0, SR = 0;
            for (int c = 0; c < C; ++c) {
                const uint32_t l = (uint32_t)((cur[c >> 2] >> (16 * (c & 3))) & 0xffffu);
                const uint32_t r = (uint32_t)S.pc[c] - l;
                SL += (uint64_t)l * l;
                SR += (uint64_t)r * r;
            }
            u128 N;
            uint64_t Dq;
            if (make_q((int64_t)i + 1, n - i - 1, SL, SR, N, Dq) && (!bv || q_greater(N, Dq, bN, bD))) {
                bv = true; bN = N; bD = Dq; bpos = i; bSL = SL; bSR = SR;
            }
        }
    }
    const int win = wave_best_lane(bv, bN, bD, bpos);
    const int src = win < 0 ? 0 : win;
    const uint64_t nlo = __shfl((uint64_t)bN, src), nhi = __shfl((uint64_t)(bN >> 64), src);
    const uint64_t dd = __shfl(bD, src), sl = __shfl(bSL, src), sr = __shfl(bSR, src);
    const int pp = __shfl(bpos, src);
    if (lane == 0) {
        S.wN[w][0] = nlo; S.wN[w][1] = nhi; S.wD[w] = win < 0 ? 0 : dd;
        S.wSL[w] = sl; S.wSR[w] = sr; S.wpos[w] = pp;
    }
    __syncthreads();
    if (tid == 0) {
        int bw = -1;
        for (int ww = 0; ww < kWavesPerBlock; ++ww) {
            if (S.wD[ww] == 0) continue;
            if (bw < 0) { bw = ww; continue; }
            const u128 a = ((u128)S.wN[ww][1] << 64) | S.wN[ww][0];
            const u128 b = ((u128)S.wN[bw][1] << 64) | S.wN[bw][0];
            if (q_greater(a, S.wD[ww], b, S.wD[bw]) ||
                (!q_greater(b, S.wD[bw], a, S.wD[ww]) && S.wpos[ww] < S.wpos[bw]))
                bw = ww;
        }
        Cand c;
        cand_invalid(c);
        c.SP = SP;
        c.proj = p;
        c.lo = kfloat((uint32_t)(keys[0] >> 32));
        if (bw >= 0) {
            const int pos = S.wpos[bw];
            c.N = ((u128)S.wN[bw][1] << 64) | S.wN[bw][0];
            c.D = S.wD[bw];
            c.SL = S.wSL[bw];
            c.SR = S.wSR[bw];
            c.pos = pos;
            c.nL = pos + 1;
            c.nR = (int32_t)(n - c.nL);
            c.thr = kfloat((uint32_t)(keys[pos] >> 32));
        }
        ((Cand*)A.ws.slots)[D.y + p] = c;
    }
    if (w == 0) write_zero_row(A, proj_global(P, v, p));
    __syncthreads();
}

template <typename T, class PS, bool ENT>
__global__ __launch_bounds__(kBlock) void k_sortblk(FindArgs A, PS P) {
    extern __shared__ __align__(16) char smem[];
    SortShared& S = *(SortShared*)smem;
    const FindWs& W = A.ws;
    const int ni = count_of(A, H_ISB, W.cap_isb);
    const int nd = count_of(A, H_DSB, W.cap_dsb);
    for (;;) {
        int it = block_dequeue(&W.hdr[H_Q_SB], &S.item);
        if (it >= ni) break;
        int2 e = W.items_sb[it];
        if (e.x >= nd) continue;
        int4 D = W.desc_sb[e.x];
        if (e.y < D.w) do_sortblock<T, PS, ENT>(A, P, D, e.y, smem);
    }
}

// ---------------------------------------------------------------------------
// host side

// the entropy criterion's table of k ln k, k = 0 .. n - 1
__global__ __launch_bounds__(kBlock) void k_flnk(double* tab, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        tab[i] = klnk(i);
}

template <typename T, class PS, bool RW, bool ENT>
static hipError_t launch_find_t(const FindArgs& a, const PS& p, const LaunchCfg& cfg, const FindStreams& st,
                                const hipEvent_t* ev) {
    const int Nc = a.n_nodes > 0 ? a.n_nodes : 1;
    int grid_plan = (Nc + kBlock - 1) / kBlock;
    if (grid_plan > 4 * cfg.n_cu) grid_plan = 4 * cfg.n_cu;
    const size_t sm = cfg.smem_main;
    const hipStream_t s = st.main;
    const bool fork = st.aux[0] && st.aux[1];
    const hipStream_t sb = fork ? st.aux[0] : s;   // big-node chain
    const hipStream_t sl = fork ? st.aux[1] : s;   // large mid nodes, then sort blocks
    hipError_t e = hipSuccess;
    auto rec = [&](int i, hipStream_t q) {
        if (ev && ev[i] && e == hipSuccess) e = hipEventRecord(ev[i], q);
    };
    auto beg = [&](int stage, hipStream_t q) { rec(2 * stage, q); };
    auto end = [&](int stage, hipStream_t q) { rec(2 * stage + 1, q); };
    rec(2 * SOF_STAGE_COUNT, s);
    beg(SOF_STAGE_PLAN, s);
    if (ENT && a.ws.cap_flnk > 0) {
        int64_t g = (a.ws.cap_flnk + kBlock - 1) / kBlock;
        if (g > 4 * cfg.n_cu) g = 4 * cfg.n_cu;
        hipLaunchKernelGGL(k_flnk, dim3((unsigned)g), dim3(kBlock), 0, s, a.ws.flnk, a.ws.cap_flnk);
    }
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, a.ws.hdr);
    hipLaunchKernelGGL((k_plan<PS>), dim3(grid_plan), dim3(kBlock), 0, s, a, p);
    hipLaunchKernelGGL((k_expand<PS>), dim3(cfg.grid_light), dim3(kBlock), 0, s, a, p);
    end(SOF_STAGE_PLAN, s);
    // The size classes are independent of each other: the big-node chain and
    // the large mid nodes run on the context's streams beside the caller's,
    // so each kernel's tail overlaps the others' work.
    if (fork && e == hipSuccess) {
        e = hipEventRecord(st.fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(sb, st.fork, 0);
        if (e == hipSuccess) e = hipStreamWaitEvent(sl, st.fork, 0);
    }
    if (e != hipSuccess) return e;
    beg(SOF_STAGE_BIG_RANGE, sb);
    hipLaunchKernelGGL((k_brange<T, PS>), dim3(cfg.grid_brange), dim3(kBlock), sm, sb, a, p);
    end(SOF_STAGE_BIG_RANGE, sb);
    beg(SOF_STAGE_BIG_MERGE, sb);
    hipLaunchKernelGGL(k_bmerge, dim3(cfg.grid_light), dim3(kBlock), 0, sb, a);
    end(SOF_STAGE_BIG_MERGE, sb);
    beg(SOF_STAGE_BIG_HIST, sb);
    hipLaunchKernelGGL((k_bhist<T, PS, RW>), dim3(cfg.grid_bhist), dim3(kBlock), sm, sb, a, p);
    end(SOF_STAGE_BIG_HIST, sb);
    beg(SOF_STAGE_BIG_SCAN, sb);
    hipLaunchKernelGGL((k_bscan<PS, RW, ENT>), dim3(cfg.grid_bscan), dim3(kBlock), sm, sb, a, p);
    end(SOF_STAGE_BIG_SCAN, sb);
    beg(SOF_STAGE_MID2, sl);
    hipLaunchKernelGGL((k_mid<T, PS, true, RW, ENT>), dim3(cfg.grid_mid2), dim3(kBlock), sm, sl, a, p);
    end(SOF_STAGE_MID2, sl);
    beg(SOF_STAGE_SORT, sl);
    hipLaunchKernelGGL((k_sortblk<T, PS, ENT>), dim3(cfg.grid_sort), dim3(kBlock), cfg.smem_sort, sl, a, p);
    end(SOF_STAGE_SORT, sl);
    beg(SOF_STAGE_MID, s);
    hipLaunchKernelGGL((k_mid<T, PS, false, RW, ENT>), dim3(cfg.grid_mid), dim3(kBlock), sm, s, a, p);
    end(SOF_STAGE_MID, s);
    beg(SOF_STAGE_SMALL, s);
    hipLaunchKernelGGL((k_small<T, PS, RW, ENT>), dim3(cfg.grid_small), dim3(kBlock), sm, s, a, p);
    end(SOF_STAGE_SMALL, s);
    if (e == hipSuccess) e = hipGetLastError();
    if (fork && e == hipSuccess) {
        e = hipEventRecord(st.join[0], sb);
        if (e == hipSuccess) e = hipEventRecord(st.join[1], sl);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, st.join[0], 0);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, st.join[1], 0);
    }
    if (e != hipSuccess) return e;
    beg(SOF_STAGE_REDUCE, s);
    hipLaunchKernelGGL(k_reduce, dim3(cfg.grid_light), dim3(kBlock), 0, s, a);
    end(SOF_STAGE_REDUCE, s);
    rec(2 * SOF_STAGE_COUNT + 1, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_find_csr(const FindArgs& a, const ProjCSR& p, const LaunchCfg& cfg, const FindStreams& s,
                           const hipEvent_t* ev) {
    const int mode = (a.bin_mode == SOF_BINS_RANDOM ? 1 : 0) | (a.criterion == SOF_CRIT_ENTROPY ? 2 : 0);
    if (a.dtype == SOF_F16) {
        switch (mode) {
        case 1: return launch_find_t<_Float16, ProjCSR, true, false>(a, p, cfg, s, ev);
        case 2: return launch_find_t<_Float16, ProjCSR, false, true>(a, p, cfg, s, ev);
        case 3: return launch_find_t<_Float16, ProjCSR, true, true>(a, p, cfg, s, ev);
        default: return launch_find_t<_Float16, ProjCSR, false, false>(a, p, cfg, s, ev);
        }
    }
    switch (mode) {
    case 1: return launch_find_t<float, ProjCSR, true, false>(a, p, cfg, s, ev);
    case 2: return launch_find_t<float, ProjCSR, false, true>(a, p, cfg, s, ev);
    case 3: return launch_find_t<float, ProjCSR, true, true>(a, p, cfg, s, ev);
    default: return launch_find_t<float, ProjCSR, false, false>(a, p, cfg, s, ev);
    }
}
hipError_t launch_find_hash(const FindArgs& a, const ProjHash& p, const LaunchCfg& cfg, const FindStreams& s,
                            const hipEvent_t* ev) {
    const int mode = (a.bin_mode == SOF_BINS_RANDOM ? 1 : 0) | (a.criterion == SOF_CRIT_ENTROPY ? 2 : 0);
    if (a.dtype == SOF_F16) {
        switch (mode) {
        case 1: return launch_find_t<_Float16, ProjHash, true, false>(a, p, cfg, s, ev);
        case 2: return launch_find_t<_Float16, ProjHash, false, true>(a, p, cfg, s, ev);
        case 3: return launch_find_t<_Float16, ProjHash, true, true>(a, p, cfg, s, ev);
        default: return launch_find_t<_Float16, ProjHash, false, false>(a, p, cfg, s, ev);
        }
    }
    switch (mode) {
    case 1: return launch_find_t<float, ProjHash, true, false>(a, p, cfg, s, ev);
    case 2: return launch_find_t<float, ProjHash, false, true>(a, p, cfg, s, ev);
    case 3: return launch_find_t<float, ProjHash, true, true>(a, p, cfg, s, ev);
    default: return launch_find_t<float, ProjHash, false, false>(a, p, cfg, s, ev);
    }
}

// resident blocks per CU of a kernel (at least 1)
static hipError_t occ(const void* f, size_t smem, int* out) {
    int b = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, f, kBlock, smem);
    *out = b > 0 ? b : 1;
    return e;
}

template <bool RW, bool ENT>
static hipError_t find_occupancy_t(int bins, int classes, int n_cu, LaunchCfg* cfg) {
    const size_t sm = find_smem_main(bins, classes, RW, ENT), ss = find_smem_sort();
    int b = 0;
    hipError_t e;
    cfg->n_cu = n_cu;
    cfg->smem_main = sm;
    cfg->smem_sort = ss;
    if ((e = occ((const void*)k_mid<float, ProjCSR, false, RW, ENT>, sm, &b)) != hipSuccess) return e;
    cfg->grid_mid = n_cu * b;
    if ((e = occ((const void*)k_mid<float, ProjCSR, true, RW, ENT>, sm, &b)) != hipSuccess) return e;
    cfg->grid_mid2 = n_cu * b;
    if ((e = occ((const void*)k_small<float, ProjCSR, RW, ENT>, sm, &b)) != hipSuccess) return e;
    cfg->grid_small = n_cu * b;
    if ((e = occ((const void*)k_sortblk<float, ProjCSR, ENT>, ss, &b)) != hipSuccess) return e;
    cfg->grid_sort = n_cu * b;
    if ((e = occ((const void*)k_brange<float, ProjCSR>, sm, &b)) != hipSuccess) return e;
    cfg->grid_brange = n_cu * b;
    if ((e = occ((const void*)k_bhist<float, ProjCSR, RW>, sm, &b)) != hipSuccess) return e;
    cfg->grid_bhist = n_cu * b;
    if ((e = occ((const void*)k_bscan<ProjCSR, RW, ENT>, sm, &b)) != hipSuccess) return e;
    cfg->grid_bscan = n_cu * b;
    cfg->grid_light = n_cu * 4;
    return hipSuccess;
}

hipError_t find_occupancy(int bins, int classes, int mode, int n_cu, LaunchCfg* cfg) {
    switch (mode & 3) {
    case 1: return find_occupancy_t<true, false>(bins, classes, n_cu, cfg);
    case 2: return find_occupancy_t<false, true>(bins, classes, n_cu, cfg);
    case 3: return find_occupancy_t<true, true>(bins, classes, n_cu, cfg);
    default: return find_occupancy_t<false, false>(bins, classes, n_cu, cfg);
    }
}

}  // namespace sof
