// sof_device.h -- device helpers shared by the split-search kernels (gfx950).
//
// Arithmetic contract (paper section 4, steps 1-3, with the precision choices
// of this library):
//  * projected value: acc = +0.0f, then acc = acc + (+/-x) per nonzero in CSR
//    order, every add correctly rounded (__fadd_rn, no contraction);
//  * equal-width bins: scale = bins / (hi - lo) correctly rounded (__fdiv_rn),
//    FLT_MAX when not finite; t = (v - lo) * scale with __fsub_rn/__fmul_rn;
//    bin = t < bins ? trunc(t) : bins - 1;
//  * Gini: maximise Q = S_L/n_L + S_R/n_R = N/D compared exactly as
//    N1*D2 > N2*D1 in unsigned 128-bit integers; split iff n*N > S_P*D.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <float.h>

namespace sof {

typedef unsigned __int128 u128;

constexpr int kWave = 64;
constexpr int kBlock = 256;          // work-group size of the persistent kernels
constexpr int kWavesPerBlock = kBlock / kWave;

// ---------------------------------------------------------------------------
// float keys that order like the floats (finite values; -0 < +0 never arises)

__device__ __forceinline__ uint32_t fkey(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float kfloat(uint32_t k) {
    uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
}

// ---------------------------------------------------------------------------
// feature loads: FP32 as is, FP16 widened exactly

__device__ __forceinline__ float ldx(const float* col, int32_t r) { return col[r]; }
__device__ __forceinline__ float ldx(const _Float16* col, int32_t r) { return (float)col[r]; }

// w * x, one FP32 rounding (exact for w = +/-1); w given as FP32 bits
__device__ __forceinline__ float weighted_term(float x, uint32_t wbits) {
    return __fmul_rn(x, __uint_as_float(wbits));
}

// ---------------------------------------------------------------------------
// bins

__device__ __forceinline__ float bin_scale(int bins, float lo, float hi) {
    float s = __fdiv_rn((float)bins, __fsub_rn(hi, lo));
    return (s <= FLT_MAX) ? s : FLT_MAX;
}
__device__ __forceinline__ int bin_index(float v, float lo, float scale, int bins) {
    float t = __fmul_rn(__fsub_rn(v, lo), scale);
    return t < (float)bins ? (int)t : bins - 1;
}
__device__ __forceinline__ float hist_threshold(float lo, float scale, int bin) {
    return __fadd_rn(lo, __fdiv_rn((float)(bin + 1), scale));
}

// ---------------------------------------------------------------------------
// wave primitives (wave64)

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        uint32_t t = __shfl_up(x, off);
        if (lane >= off) x += t;
    }
    return x;
}

// Wave-aggregated allocation from K counters at once (every lane calls):
// lane l asks cnt[k] entries of counter hdr[ctr[k]] and gets base[k], the
// start of its entries; a wave's entries of one counter are contiguous in
// lane order.  The K atomics are one instruction, issued by lanes 0..K-1, so
// the wave waits for one round trip instead of K.
template <int K>
__device__ __forceinline__ void wave_alloc_n(int32_t* hdr, const int (&ctr)[K], const int (&cnt)[K],
                                             int (&base)[K]) {
    static_assert(K <= kWave, "one counter per lane");
    const int lane = lane_id();
    uint32_t incl[K];
    int my_ctr = 0;
    uint32_t my_tot = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        incl[k] = wave_incl_scan((uint32_t)cnt[k]);
        const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl[k], kWave - 1);
        if (lane == k) { my_ctr = ctr[k]; my_tot = tot; }
    }
    int b = 0;
    if (lane < K && my_tot) b = atomicAdd(&hdr[my_ctr], (int)my_tot);
#pragma unroll
    for (int k = 0; k < K; ++k) base[k] = __builtin_amdgcn_readlane(b, k) + (int)(incl[k] - (uint32_t)cnt[k]);
}

__device__ __forceinline__ float wave_min(float x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = fminf(x, __shfl_xor(x, off));
    return x;
}
__device__ __forceinline__ float wave_max(float x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = fmaxf(x, __shfl_xor(x, off));
    return x;
}
__device__ __forceinline__ double wave_max_d(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off));
    return x;
}
__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// ---------------------------------------------------------------------------
// DPP (data-parallel primitives) cross-lane steps of the GFX9 family.  Each
// reads a neighbouring lane of the same 16-lane row without going through the
// LDS crossbar.  update_dpp(old, src, ctrl, row_mask, bank_mask, bound_ctrl):
// lanes whose source is outside the row read 0 when bound_ctrl is set;
// lanes of rows disabled by row_mask keep `old`.

enum : int {
    kDppXor1 = 0xB1,          // quad_perm [1,0,3,2]
    kDppXor2 = 0x4E,          // quad_perm [2,3,0,1]
    kDppShr1 = 0x111,         // row_shr:1
    kDppShr2 = 0x112,
    kDppShr4 = 0x114,
    kDppShr8 = 0x118,
    kDppRowMirror = 0x140,    // lane i <- lane 15-i of the row
    kDppHalfMirror = 0x141,   // lane i <- lane 7-i of the half row
    kDppBcast15 = 0x142,      // lane 15 of each row -> the next row
    kDppBcast31 = 0x143,      // lane 31 -> rows 2 and 3
};

template <int kCtrl>
__device__ __forceinline__ uint32_t dpp_u(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kCtrl, 0xf, 0xf, true);
}
template <int kCtrl>
__device__ __forceinline__ float dpp_f(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kCtrl, 0xf, 0xf, true));
}

// inclusive prefix sum over the 64 lanes (exact for integers; for floats
// holding integers below 2^24 as well)
__device__ __forceinline__ uint32_t wave_scan_u(uint32_t x) {
    x += dpp_u<kDppShr1>(x);
    x += dpp_u<kDppShr2>(x);
    x += dpp_u<kDppShr4>(x);
    x += dpp_u<kDppShr8>(x);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppBcast15, 0xa, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppBcast31, 0xc, 0xf, false);
    return x;
}
__device__ __forceinline__ float wave_scan_f(float x) {
    x += dpp_f<kDppShr1>(x);
    x += dpp_f<kDppShr2>(x);
    x += dpp_f<kDppShr4>(x);
    x += dpp_f<kDppShr8>(x);
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kDppBcast15, 0xa, 0xf, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kDppBcast31, 0xc, 0xf, false));
    return x;
}

// Butterfly over each 16-lane row (every lane ends with its row's result),
// then the four row results read with readlane: the wave result, uniform.
__device__ __forceinline__ float wave_min_f(float x) {
    x = fminf(x, dpp_f<kDppXor1>(x));
    x = fminf(x, dpp_f<kDppXor2>(x));
    x = fminf(x, dpp_f<kDppHalfMirror>(x));
    x = fminf(x, dpp_f<kDppRowMirror>(x));
    const int b = __float_as_int(x);
    return fminf(fminf(__int_as_float(__builtin_amdgcn_readlane(b, 0)), __int_as_float(__builtin_amdgcn_readlane(b, 16))),
                 fminf(__int_as_float(__builtin_amdgcn_readlane(b, 32)), __int_as_float(__builtin_amdgcn_readlane(b, 48))));
}
__device__ __forceinline__ float wave_max_f(float x) {
    x = fmaxf(x, dpp_f<kDppXor1>(x));
    x = fmaxf(x, dpp_f<kDppXor2>(x));
    x = fmaxf(x, dpp_f<kDppHalfMirror>(x));
    x = fmaxf(x, dpp_f<kDppRowMirror>(x));
    const int b = __float_as_int(x);
    return fmaxf(fmaxf(__int_as_float(__builtin_amdgcn_readlane(b, 0)), __int_as_float(__builtin_amdgcn_readlane(b, 16))),
                 fmaxf(__int_as_float(__builtin_amdgcn_readlane(b, 32)), __int_as_float(__builtin_amdgcn_readlane(b, 48))));
}
__device__ __forceinline__ uint32_t wave_sum_u(uint32_t x) {
    x += dpp_u<kDppXor1>(x);
    x += dpp_u<kDppXor2>(x);
    x += dpp_u<kDppHalfMirror>(x);
    x += dpp_u<kDppRowMirror>(x);
    const int b = (int)x;
    return (uint32_t)__builtin_amdgcn_readlane(b, 0) + (uint32_t)__builtin_amdgcn_readlane(b, 16) +
           (uint32_t)__builtin_amdgcn_readlane(b, 32) + (uint32_t)__builtin_amdgcn_readlane(b, 48);
}

// bits of lanes strictly below / up to and including this lane
__device__ __forceinline__ uint64_t lanes_le_mask() {
    const int lane = lane_id();
    return lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
}

// ---------------------------------------------------------------------------
// candidates

// Q1 > Q2 with Q = N / D, D > 0.  N <= 2^70 and D <= 2^46 for n <= 2^24, so
// both products fit in 128 bits.
__device__ __forceinline__ bool q_greater(u128 n1, uint64_t d1, u128 n2, uint64_t d2) {
    return n1 * (u128)d2 > n2 * (u128)d1;
}

// One candidate boundary, with what the node record needs.
struct Cand {
    u128     N;       // S_L*n_R + S_R*n_L
    uint64_t D;       // n_L*n_R; 0 = invalid
    uint64_t SL, SR, SP;
    int32_t  pos;     // bin or sorted position
    int32_t  proj;    // node-local projection
    float    thr, lo, scale;
    int32_t  nL, nR;
};
static_assert(sizeof(Cand) == 80, "slot layout");

__device__ __forceinline__ void cand_invalid(Cand& c) {
    c.N = 0; c.D = 0; c.SL = c.SR = c.SP = 0; c.pos = -1; c.proj = -1;
    c.thr = c.lo = c.scale = 0.f; c.nL = c.nR = 0;
}

// a strictly better than b; invalid (D == 0) is worse than anything valid
__device__ __forceinline__ bool cand_better(const Cand& a, const Cand& b) {
    if (a.D == 0) return false;
    if (b.D == 0) return true;
    return q_greater(a.N, a.D, b.N, b.D);
}

// Lane holding the best (largest Q, then lowest pos) valid candidate, or -1.
// Every lane returns the same value.
__device__ __forceinline__ int wave_best_lane(bool valid, u128 N, uint64_t D, int32_t pos) {
    uint64_t nlo = (uint64_t)N, nhi = (uint64_t)(N >> 64);
    uint64_t d = valid ? D : 1ull;
    if (!valid) { nlo = 0; nhi = 0; }
    int32_t bp = valid ? pos : 0x7fffffff;
    int32_t bl = lane_id();
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        uint64_t olo = __shfl_xor(nlo, off), ohi = __shfl_xor(nhi, off), od = __shfl_xor(d, off);
        int32_t op = __shfl_xor(bp, off), ol = __shfl_xor(bl, off);
        u128 on = ((u128)ohi << 64) | olo, mn = ((u128)nhi << 64) | nlo;
        bool take = q_greater(on, od, mn, d) || (!q_greater(mn, d, on, od) && op < bp);
        if (take) { nlo = olo; nhi = ohi; d = od; bp = op; bl = ol; }
    }
    return bp == 0x7fffffff ? -1 : bl;
}

// Evaluate the boundary with left counts summarised by n_L, S_L and right
// summarised by n_R, S_R.
__device__ __forceinline__ bool make_q(int64_t nL, int64_t nR, uint64_t SL, uint64_t SR, u128& N,
                                       uint64_t& D) {
    if (nL < 1 || nR < 1) return false;
    N = (u128)SL * (u128)(uint64_t)nR + (u128)SR * (u128)(uint64_t)nL;
    D = (uint64_t)nL * (uint64_t)nR;
    return true;
}

// round-to-nearest u128 -> float
__device__ __forceinline__ float u128_to_float(u128 x) {
    uint64_t hi = (uint64_t)(x >> 64), lo = (uint64_t)x;
    if (hi == 0) return (float)lo;
    int sh = 64 - __clzll((long long)hi);
    uint64_t m = (uint64_t)(x >> sh);
    if (lo & ((1ull << sh) - 1ull)) m |= 1ull;   // sticky bit below the rounding point
    return ldexpf((float)m, sh);
}

// ---------------------------------------------------------------------------
// Entropy criterion helpers.  f(k) = k ln k in binary64, with the natural log
// of an integer built from IEEE basic operations only (each correctly
// rounded, so any implementation of the same sequence gets the same bits):
// k = m 2^e with m in [sqrt(2)/2, sqrt(2)), ln m = 2 atanh(s) with
// s = (m - 1) / (m + 1), summed as 2 (s + s^3/3 + ... + s^25/25)
// (Abramowitz and Stegun 4.1.27; |s| <= 0.172, first omitted term below 2^-60
// of the sum).
__device__ __forceinline__ double ln_int(int64_t k) {
    int e = 63 - __clzll((long long)k);          // k >= 1: m = k 2^-e in [1, 2), exact
    double m = ldexp((double)k, -e);
    if (m > 1.4142135623730951) {
        m = __dmul_rn(m, 0.5);
        ++e;
    }
    const double s = __ddiv_rn(__dsub_rn(m, 1.0), __dadd_rn(m, 1.0));
    const double s2 = __dmul_rn(s, s);
    double t = s, sum = s;
#pragma unroll
    for (int j = 1; j <= 12; ++j) {
        t = __dmul_rn(t, s2);
        sum = __dadd_rn(sum, __ddiv_rn(t, (double)(2 * j + 1)));
    }
    return __dadd_rn(__dmul_rn((double)e, 0.69314718055994530942), __dmul_rn(2.0, sum));
}
__device__ __forceinline__ double klnk(int64_t k) { return k <= 0 ? 0.0 : __dmul_rn((double)k, ln_int(k)); }

// Order-preserving map of a (non-NaN) double to an unsigned key, and back:
// an entropy candidate keeps key(E) in N and 1 in D, so the exact (N, D)
// comparisons below order it by E.
__device__ __forceinline__ uint64_t dkey(double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double dkey_inv(uint64_t k) {
    return __longlong_as_double((long long)((k >> 63) ? (k & 0x7fffffffffffffffull) : ~k));
}
__device__ __forceinline__ double bits_d(uint64_t b) { return __longlong_as_double((long long)b); }
__device__ __forceinline__ uint64_t d_bits(double x) { return (uint64_t)__double_as_longlong(x); }

// The node record of the best candidate (n = node size).
struct SplitRec {
    int32_t proj, kind, bin;
    float threshold, lo, scale;
    int32_t n_left, n_right, flags;
    float gain;
};
static_assert(sizeof(SplitRec) == 40, "sof_split layout");

// Gini: split iff n N > S_P D, gain (n N - S_P D) / (n^2 D).  Entropy (N =
// key of E, SL / SR / SP = bits of sum f(l_c), sum f(r_c), sum f(P_c)): gain
// ((f(n) - sum f(P_c)) + E) / n, split iff it exceeds 1e-12.
__device__ __forceinline__ void write_record(SplitRec* out, const Cand& b, int kind, int32_t n,
                                             bool entropy = false) {
    SplitRec r;
    bool split = false;
    u128 lhs = 0, rhs = 0;
    double ig = 0.0;
    if (b.D != 0 && entropy) {
        ig = __ddiv_rn(__dadd_rn(__dsub_rn(klnk(n), bits_d(b.SP)), dkey_inv((uint64_t)b.N)), (double)n);
        split = ig > 1e-12;
    } else if (b.D != 0) {
        lhs = (u128)(uint64_t)n * b.N;
        rhs = (u128)b.SP * (u128)b.D;
        split = lhs > rhs;
    }
    if (!split) {
        r.proj = -1; r.kind = kind; r.bin = -1; r.threshold = 0.f; r.lo = 0.f; r.scale = 0.f;
        r.n_left = n; r.n_right = 0; r.flags = 0; r.gain = 0.f;
    } else {
        r.proj = b.proj; r.kind = kind; r.bin = b.pos; r.threshold = b.thr; r.lo = b.lo;
        r.scale = b.scale; r.n_left = b.nL; r.n_right = b.nR;
        if (entropy) {
            r.flags = (bits_d(b.SL) == klnk(b.nL) ? 1 : 0) | (bits_d(b.SR) == klnk(b.nR) ? 2 : 0);
            r.gain = (float)ig;
        } else {
            r.flags = (b.SL == (uint64_t)b.nL * (uint64_t)b.nL ? 1 : 0) |
                      (b.SR == (uint64_t)b.nR * (uint64_t)b.nR ? 2 : 0);
            u128 den = (u128)((uint64_t)n * (uint64_t)n) * (u128)b.D;
            r.gain = __fdiv_rn(u128_to_float(lhs - rhs), u128_to_float(den));
        }
    }
    *out = r;
}

}  // namespace sof
