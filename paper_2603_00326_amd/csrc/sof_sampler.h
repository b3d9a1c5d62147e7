// sof_sampler.h -- the counter-based projection sampler of tree growth, one
// definition for the split search, the partition and the node records, so
// the three draw the same projection bit for bit.
//
// A projection of node (tree, level, pos) with index p is a function of
// those four numbers and the seed only.  Every random number is one output
// of SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) at a counter that packs
// (tree, level, pos, p, draw); independent streams use seeds xor-ed with
// fixed constants.
//
// Two laws for the number of nonzeros z_p (Method, projection matrix; the
// appendix on Floyd's sampling):
//   SOF_SAMPLER_FIXED    z_p = z, the same for every projection;
//   SOF_SAMPLER_DENSITY  every feature enters independently with probability
//                        z/d, so z_p ~ Binomial(d, z/d) (0 included), drawn by
//                        inversion in binary64 and capped at 16.
// The z_p features are then distinct draws by Floyd's algorithm (Bentley and
// Floyd, CACM 1987), stored ascending.  Two laws for the weights:
//   SOF_WEIGHTS_SIGN     +1 or -1 with equal probability;
//   SOF_WEIGHTS_UNIFORM  (2m + 1 - 2^24) / 2^24 for m uniform on 0..2^24-1:
//                        symmetric on (-1, 1), never 0, exact in FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sof.h"
#include "sof_device.h"

namespace sof {

struct SampSpec {
    uint64_t seed;
    int32_t d, z, mode, wmode;
};

constexpr uint64_t kSeedNnz = 0x6A09E667F3BCC909ull;
constexpr uint64_t kSeedWeight = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ uint64_t samp_mix(uint64_t seed, uint64_t c) {
    uint64_t z = seed + c * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// tree (any), level (6 bits), pos (24 bits), p (10 bits), draw (4 bits)
__device__ __forceinline__ uint64_t samp_counter(int tree, int level, int pos, int p, int draw) {
    uint64_t c = (uint64_t)tree * 64u + (uint64_t)level;
    c = (c << 24) + (uint64_t)pos;
    c = (c << 10) + (uint64_t)p;
    return (c << 4) + (uint64_t)draw;
}

// Number of nonzeros of the projection.  Density law: with pi = z/d,
// q = 1 - pi and r = pi/q, P(0) = q^d (binary powering, low bit first) and
// P(k+1) = (P(k) * ((d-k)/(k+1))) * r; z_p is the least k with
// u < P(0) + ... + P(k), u = (top 53 bits of the draw) / 2^53, at most
// min(d, 16); every operation is one correctly rounded binary64 operation.
__device__ __forceinline__ int samp_nnz(const SampSpec& s, int tree, int level, int pos, int p) {
    if (s.mode != SOF_SAMPLER_DENSITY) return s.z;
    const int cap = s.d < SOF_MAX_NNZ ? s.d : SOF_MAX_NNZ;
    if (s.z >= s.d) return cap;
    const double pi = __ddiv_rn((double)s.z, (double)s.d);
    const double q = __dsub_rn(1.0, pi);
    const double r = __ddiv_rn(pi, q);
    double pk = 1.0, b = q;
    for (int e = s.d; e != 0; e >>= 1) {
        if (e & 1) pk = __dmul_rn(pk, b);
        b = __dmul_rn(b, b);
    }
    const uint64_t h = samp_mix(s.seed ^ kSeedNnz, samp_counter(tree, level, pos, p, 0));
    const double u = __dmul_rn((double)(h >> 11), 0x1.0p-53);
    double cdf = pk;
    int k = 0;
    while (k < cap && u >= cdf) {
        pk = __dmul_rn(__dmul_rn(pk, __ddiv_rn((double)(s.d - k), (double)(k + 1))), r);
        cdf = __dadd_rn(cdf, pk);
        ++k;
    }
    return k;
}

// Floyd's draw j of z (j = 0..z-1): a proposal t uniform on [0, d-z+j] by
// multiply-shift of the output's top 32 bits; if t was taken by an earlier
// draw, the draw takes d-z+j instead.
__device__ __forceinline__ int samp_proposal(const SampSpec& s, int z, int j, int tree, int level, int pos,
                                             int p) {
    const uint32_t top = (uint32_t)(s.d - z + j) + 1u;
    const uint64_t r = samp_mix(s.seed, samp_counter(tree, level, pos, p, j));
    return (int)(((r >> 32) * (uint64_t)top) >> 32);
}

// Weight of the nonzero of rank `rank` (features ascending) as FP32 bits.
// Signs: bit `rank` of draw 15 for the fixed law (z <= 15 keeps draw 15 free),
// of the weight stream's draw 0 for the density law.
__device__ __forceinline__ uint32_t samp_weight_bits(const SampSpec& s, int tree, int level, int pos, int p,
                                                     int rank) {
    if (s.wmode == SOF_WEIGHTS_UNIFORM) {
        const uint64_t h = samp_mix(s.seed ^ kSeedWeight, samp_counter(tree, level, pos, p, rank));
        const int32_t m = (int32_t)(h >> 40);
        return __float_as_uint((float)(2 * m + 1 - (1 << 24)) * 0x1.0p-24f);
    }
    const uint64_t sg = s.mode == SOF_SAMPLER_DENSITY
                            ? samp_mix(s.seed ^ kSeedWeight, samp_counter(tree, level, pos, p, 0))
                            : samp_mix(s.seed, samp_counter(tree, level, pos, p, 15));
    return ((sg >> rank) & 1ull) ? 0xbf800000u : 0x3f800000u;
}

// Floyd's draws by one converged wave: lane j < z makes draw j; on return
// lane j holds draw j's feature in `mine` and its rank among the z features
// in `rank` (lanes >= z hold unspecified values).  z is wave-uniform.
__device__ __forceinline__ void samp_wave(const SampSpec& s, int z, int tree, int level, int pos, int p,
                                          int& mine, int& rank) {
    const int lane = lane_id();
    int t = lane < z ? samp_proposal(s, z, lane, tree, level, pos, p) : 0;
    mine = t;
    for (int j = 0; j < z; ++j) {
        const int cj = __shfl(t, j);
        const bool taken = __ballot(lane < j && mine == cj) != 0ull;
        if (lane == j) mine = taken ? s.d - z + j : cj;
    }
    rank = 0;
    for (int i = 0; i < z; ++i) rank += (__shfl(mine, i) < mine) ? 1 : 0;
}

// The whole projection by one thread: features ascending in f[0..z-1],
// weight bits in w[0..z-1]; returns z.
__device__ __forceinline__ int samp_thread(const SampSpec& s, int tree, int level, int pos, int p, int32_t* f,
                                           uint32_t* w) {
    const int z = samp_nnz(s, tree, level, pos, p);
    int32_t c[SOF_MAX_NNZ];
    for (int j = 0; j < z; ++j) {
        const int t = samp_proposal(s, z, j, tree, level, pos, p);
        bool taken = false;
        for (int i = 0; i < j; ++i) taken |= c[i] == t;
        c[j] = taken ? s.d - z + j : t;
    }
    for (int i = 1; i < z; ++i) {
        const int key = c[i];
        int m = i - 1;
        while (m >= 0 && c[m] > key) { c[m + 1] = c[m]; --m; }
        c[m + 1] = key;
    }
    for (int q = 0; q < z; ++q) {
        f[q] = c[q];
        w[q] = samp_weight_bits(s, tree, level, pos, p, q);
    }
    return z;
}

}  // namespace sof
