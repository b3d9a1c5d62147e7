/*
 * sof_oracle.c -- reference CPU implementation of per-node split search for
 * sparse oblique forests.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark; never by the GPU library, with which it shares
 * no code.  Plain, slow and meant to be checked by eye against the paper.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 * x86-64 evaluates float expressions in binary32 (FLT_EVAL_METHOD 0), so every
 * float operation below is one correctly rounded IEEE operation.
 *
 * What is computed, step by step (paper section 4, steps 1-3):
 *
 *  1. Projection ("build the feature by combining the active samples of the
 *     data columns for the non-zero offsets and apply weights"): for sample r,
 *     acc = +0.0f, then acc = acc + (w_j * x[f_j][r]) for the nonzeros j in CSR
 *     order, each product and each add one FP32 rounding (no fused
 *     multiply-add).  With w_j = +/-1 every product is exact.  FP16 storage is
 *     widened exactly first.
 *  2. Node range: lo = min, hi = max of the projected values of the node.
 *  3. Histogram ("assign samples to bins and count the class instances in
 *     each bin") with equal-width bins over [lo, hi] (the paper notes equal
 *     width needs only a few arithmetic operations):
 *        scale = B / (hi - lo)           (each op correctly rounded; a result
 *                                          that is not finite becomes FLT_MAX)
 *        t     = (v - lo) * scale
 *        bin   = t < B ? trunc(t) : B - 1
 *     Candidate split after bin b (b = 0..B-2): left = samples with bin <= b.
 *  3''. Random-width bins (the Introduction's footnote: bin boundaries at
 *     random-width intervals; the paper gives no sampling rule, so this one is
 *     a reading): for projection q (its index in the call) the B bin widths are
 *     integers g_j = 1 + (bits 63..48 of SplitMix64 output 256 q + j of the
 *     stream started at the seed), G_i = g_0 + ... + g_{i-1} (exact, G_B <=
 *     2^24), and boundary i = 1..B-1 is t_i = lo + (G_i / G_B) * (hi - lo),
 *     each operation rounded once.  A value's bin is the number of boundaries
 *     <= v (std::upper_bound), so bin(v) <= b iff v < t_{b+1}: the split keeps
 *     t_{b+1} as its threshold.
 *  3'. Sort path (section 4.1: sorting for low-cardinality nodes): sort the
 *     projected values; candidates between sorted positions i and i+1 where
 *     v_(i) < v_(i+1), left = first i+1 samples, threshold v_(i).
 *     Node v takes the sort path iff n_v < min(T, OR_SORT_LIMIT + 1).
 *  4. Criterion ("evaluate a splitting criterion at each split and return the
 *     boundary that best separates the data"): Gini.  For left counts l_c,
 *     right counts r_c, with S_L = sum l_c^2, S_R = sum r_c^2, a candidate is
 *     valid iff n_L >= 1 and n_R >= 1, and the Gini decrease is monotone in
 *     Q = S_L/n_L + S_R/n_R = N/D, N = S_L*n_R + S_R*n_L, D = n_L*n_R.
 *     Candidates are compared exactly (N1*D2 > N2*D1 in 128-bit integers) in
 *     the order projection ascending, then bin / sorted position ascending;
 *     a candidate replaces the incumbent only when strictly better, so ties go
 *     to the lowest projection, then the lowest bin or position.
 *     The node splits iff the best candidate has a positive decrease,
 *     n*N > S_P*D with S_P = sum of squared parent counts; the reported gain
 *     is (n*N - S_P*D) / (n^2 * D) in binary64.
 *  4'. Entropy criterion (information gain, YDF's own, Method step 3): with
 *     f(k) = k ln k, maximising the gain H(P) - n_L/n H(L) - n_R/n H(R) is
 *     maximising E = sum_c f(l_c) + sum_c f(r_c) - f(n_L) - f(n_R).  E is
 *     evaluated in binary64 with a natural logarithm built from IEEE basic
 *     operations only (or_ln_int below), the sums taken over c in ascending
 *     order, so that an implementation performing the same operations gets the
 *     same bits and the same argmax; a candidate replaces the incumbent only on
 *     a strictly larger E.  The gain is ((f(n) - sum_c f(P_c)) + E) / n and
 *     the node splits iff it exceeds 1e-12 (rounding stays below 1e-13 for
 *     n <= 2^24).
 */
#include "sof_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------ */
/* storage                                                                   */
/* ------------------------------------------------------------------------ */

float or_half_to_float(uint16_t h)
{
    /* IEEE 754 binary16: 1 sign bit, 5 exponent bits (bias 15), 10 fraction bits. */
    uint32_t s = (h >> 15) & 1u, e = (h >> 10) & 0x1fu, m = h & 0x3ffu;
    float mag;
    if (e == 0)
        mag = ldexpf((float)m, -24);                 /* subnormal: m * 2^-24 */
    else if (e == 31)
        mag = m ? NAN : INFINITY;
    else
        mag = ldexpf((float)(m | 0x400u), (int)e - 25); /* (1024 + m) * 2^(e-25) */
    return s ? -mag : mag;
}

static float load_x(const void* x, int dtype, int64_t ld, int32_t f, int32_t r)
{
    int64_t at = (int64_t)f * ld + r;
    if (dtype == OR_F16)
        return or_half_to_float(((const uint16_t*)x)[at]);
    return ((const float*)x)[at];
}

/* ------------------------------------------------------------------------ */
/* step 1: projection                                                        */
/* ------------------------------------------------------------------------ */

float or_project_value(const void* x, int dtype, int64_t ld, const int32_t* feat,
                       const float* w, int z, int32_t row)
{
    float acc = 0.0f;
    for (int j = 0; j < z; ++j) {
        float term = w[j] * load_x(x, dtype, ld, feat[j], row);
        acc = acc + term;
    }
    return acc;
}

void or_project(const void* x, int dtype, int64_t ld, int32_t n_nodes,
                const int32_t* node_offsets, const int32_t* sample_idx,
                const int32_t* proj_offsets, const int32_t* nz_offsets,
                const int32_t* nz_feature, const float* nz_weight, float* out)
{
    int64_t base = 0;
    for (int32_t v = 0; v < n_nodes; ++v) {
        int32_t s0 = node_offsets[v], n = node_offsets[v + 1] - s0;
        for (int32_t q = proj_offsets[v]; q < proj_offsets[v + 1]; ++q) {
            int32_t j0 = nz_offsets[q], z = nz_offsets[q + 1] - j0;
            for (int32_t i = 0; i < n; ++i)
                out[base + i] = or_project_value(x, dtype, ld, nz_feature + j0, nz_weight + j0, z,
                                                 sample_idx[s0 + i]);
            base += n;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* steps 2-3: range and equal-width bins                                     */
/* ------------------------------------------------------------------------ */

float or_bin_scale(int n_bins, float lo, float hi)
{
    float width = hi - lo;
    float s = (float)n_bins / width;
    if (!(s <= FLT_MAX))
        s = FLT_MAX;
    return s;
}

int or_bin_index(float v, float lo, float scale, int n_bins)
{
    float d = v - lo;
    float t = d * scale;
    return t < (float)n_bins ? (int)t : n_bins - 1;
}

/* Random-width boundaries t[0..B-2] of projection q (step 3'' above). */
void or_rw_boundaries(uint64_t seed, int64_t q, int n_bins, float lo, float hi, float* t)
{
    uint32_t G[257];
    G[0] = 0;
    for (int j = 0; j < n_bins; ++j)
        G[j + 1] = G[j] + 1u + (uint32_t)(or_hash(seed, (uint64_t)q * 256u + (uint64_t)j) >> 48);
    float width = hi - lo;
    float total = (float)G[n_bins];
    for (int i = 1; i < n_bins; ++i) {
        float r = (float)G[i] / total;
        float off = r * width;
        t[i - 1] = lo + off;
    }
}

/* Random-width bin of v: how many of the B-1 (ascending) boundaries are <=
 * v, i.e. std::upper_bound's index, by binary search. */
int or_rw_bin(const float* t, int n_bins, float v)
{
    int lo = 0, hi = n_bins - 1;
    while (lo < hi) {
        int mid = lo + (hi - lo) / 2;
        if (t[mid] <= v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

/* ------------------------------------------------------------------------ */
/* step 4: exact candidate comparison                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    int valid;
    int32_t pos;
    float thr, lo, scale;
    u128 N;
    uint64_t D;
    int64_t nL, nR;
    uint64_t SL, SR;
    double E, FL, FR;   /* entropy criterion: score, sum f(l_c), sum f(r_c) */
} cand_t;

/* Natural logarithm of an integer 1 <= k < 2^53 in binary64 by a fixed
 * sequence of IEEE operations: k = m 2^e with m in [sqrt(2)/2, sqrt(2)) (exact
 * halvings), then ln m = 2 atanh(s), s = (m - 1) / (m + 1), summed as
 * 2 (s + s^3/3 + ... + s^25/25) (Abramowitz and Stegun 4.1.27); |s| <= 0.172,
 * so the first omitted term is below 2^-60 of the sum. */
double or_ln_int(int64_t k)
{
    int e = 0;
    double m = (double)k;
    while (m >= 2.0) {
        m = m * 0.5;
        ++e;
    }
    if (m > 1.4142135623730951) {
        m = m * 0.5;
        ++e;
    }
    double s = (m - 1.0) / (m + 1.0);
    double s2 = s * s;
    double t = s, sum = s;
    for (int j = 1; j <= 12; ++j) {
        t = t * s2;
        sum = sum + t / (double)(2 * j + 1);
    }
    double a = (double)e * 0.69314718055994530942;
    double b = 2.0 * sum;
    return a + b;
}

/* f(k) = k ln k, f(0) = 0. */
double or_klnk(int64_t k)
{
    if (k <= 0)
        return 0.0;
    return (double)k * or_ln_int(k);
}

static void consider_entropy(cand_t* best, const int64_t* l, const int64_t* parent, int C, int64_t n,
                             int32_t pos, float thr, float lo, float scale)
{
    int64_t nL = 0;
    double FL = 0.0, FR = 0.0;
    for (int c = 0; c < C; ++c) {
        nL += l[c];
        FL = FL + or_klnk(l[c]);
        FR = FR + or_klnk(parent[c] - l[c]);
    }
    int64_t nR = n - nL;
    if (nL < 1 || nR < 1)
        return;
    double E = ((FL + FR) - or_klnk(nL)) - or_klnk(nR);
    if (best->valid && !(E > best->E))
        return;
    best->valid = 1;
    best->pos = pos;
    best->thr = thr;
    best->lo = lo;
    best->scale = scale;
    best->E = E;
    best->FL = FL;
    best->FR = FR;
    best->nL = nL;
    best->nR = nR;
}

/* N1/D1 > N2/D2 with both denominators positive. */
static int q_greater(u128 N1, uint64_t D1, u128 N2, uint64_t D2)
{
    return N1 * (u128)D2 > N2 * (u128)D1;
}

static void consider_gini(cand_t* best, const int64_t* l, const int64_t* parent, int C, int64_t n,
                          int32_t pos, float thr, float lo, float scale);
static void consider(cand_t* best, const int64_t* l, const int64_t* parent, int C, int64_t n,
                     int32_t pos, float thr, float lo, float scale, int criterion)
{
    if (criterion == OR_CRIT_ENTROPY)
        consider_entropy(best, l, parent, C, n, pos, thr, lo, scale);
    else
        consider_gini(best, l, parent, C, n, pos, thr, lo, scale);
}

static void consider_gini(cand_t* best, const int64_t* l, const int64_t* parent, int C, int64_t n,
                          int32_t pos, float thr, float lo, float scale)
{
    int64_t nL = 0;
    uint64_t SL = 0, SR = 0;
    for (int c = 0; c < C; ++c) {
        int64_t r = parent[c] - l[c];
        nL += l[c];
        SL += (uint64_t)(l[c] * l[c]);
        SR += (uint64_t)(r * r);
    }
    int64_t nR = n - nL;
    if (nL < 1 || nR < 1)
        return;
    u128 N = (u128)SL * (u128)(uint64_t)nR + (u128)SR * (u128)(uint64_t)nL;
    uint64_t D = (uint64_t)nL * (uint64_t)nR;
    if (best->valid && !q_greater(N, D, best->N, best->D))
        return;
    best->valid = 1;
    best->pos = pos;
    best->thr = thr;
    best->lo = lo;
    best->scale = scale;
    best->N = N;
    best->D = D;
    best->nL = nL;
    best->nR = nR;
    best->SL = SL;
    best->SR = SR;
}

typedef struct {
    float v;
    int32_t y;
} vy_t;

static int cmp_vy(const void* a, const void* b)
{
    const vy_t* p = (const vy_t*)a;
    const vy_t* q = (const vy_t*)b;
    if (p->v < q->v) return -1;
    if (p->v > q->v) return 1;
    return (p->y > q->y) - (p->y < q->y);
}

static int effective_threshold(int32_t T)
{
    return T > OR_SORT_LIMIT + 1 ? OR_SORT_LIMIT + 1 : T;
}

/* Best candidate of projection q of node v (both paths). */
static void eval_projection(const void* x, int dtype, int64_t ld, const int32_t* y, int C,
                            const int32_t* idx, int32_t n, const int64_t* parent,
                            const int32_t* feat, const float* w, int z, int B, int sort_path,
                            int bin_mode, uint64_t bin_seed, int64_t q, int criterion,
                            cand_t* best, int32_t* hist_row, int32_t bins_stride)
{
    memset(best, 0, sizeof(*best));
    float* v = (float*)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
    float lo = INFINITY, hi = -INFINITY;
    for (int32_t i = 0; i < n; ++i) {
        v[i] = or_project_value(x, dtype, ld, feat, w, z, idx[i]);
        if (v[i] < lo) lo = v[i];
        if (v[i] > hi) hi = v[i];
    }
    int64_t* l = (int64_t*)calloc((size_t)C, sizeof(int64_t));
    if (!sort_path) {
        float scale = or_bin_scale(B, lo, hi);
        float t[256];
        if (bin_mode == OR_BINS_RANDOM)
            or_rw_boundaries(bin_seed, q, B, lo, hi, t);
        int64_t* H = (int64_t*)calloc((size_t)B * C, sizeof(int64_t));
        for (int32_t i = 0; i < n; ++i) {
            int b = bin_mode == OR_BINS_RANDOM ? or_rw_bin(t, B, v[i]) : or_bin_index(v[i], lo, scale, B);
            H[(int64_t)b * C + y[idx[i]]] += 1;
        }
        if (hist_row)
            for (int b = 0; b < B; ++b)
                for (int c = 0; c < C; ++c)
                    hist_row[(int64_t)b * C + c] = (int32_t)H[(int64_t)b * C + c];
        for (int b = 0; b + 1 < B; ++b) {
            for (int c = 0; c < C; ++c)
                l[c] += H[(int64_t)b * C + c];
            float thr = bin_mode == OR_BINS_RANDOM ? t[b] : lo + ((float)(b + 1) / scale);
            consider(best, l, parent, C, n, b, thr, lo, scale, criterion);
        }
        free(H);
    } else {
        vy_t* s = (vy_t*)malloc(sizeof(vy_t) * (size_t)(n > 0 ? n : 1));
        for (int32_t i = 0; i < n; ++i) {
            s[i].v = v[i];
            s[i].y = y[idx[i]];
        }
        qsort(s, (size_t)n, sizeof(vy_t), cmp_vy);
        for (int32_t i = 0; i + 1 < n; ++i) {
            l[s[i].y] += 1;
            if (s[i].v < s[i + 1].v)
                consider(best, l, parent, C, n, i, s[i].v, lo, 0.0f, criterion);
        }
        free(s);
        (void)bins_stride;
    }
    free(l);
    free(v);
}

static void no_split(or_split* o, int kind, int32_t n)
{
    memset(o, 0, sizeof(*o));
    o->proj = -1;
    o->kind = kind;
    o->bin = -1;
    o->n_left = n;
    o->n_right = 0;
}

/* bin_keys (optional): the random-width width-stream key of every projection
 * (forest growth keys a drawn projection by its tree position); NULL keys
 * projection q by q, its index in the call. */
static int find_splits_keyed(const void* x, int dtype, int64_t ld, const int32_t* y, int32_t C,
                             int32_t n_nodes, const int32_t* node_offsets, const int32_t* sample_idx,
                             const int32_t* proj_offsets, const int32_t* nz_offsets,
                             const int32_t* nz_feature, const float* nz_weight,
                             const int32_t* node_bins, int32_t bins, int32_t sort_threshold,
                             int32_t bin_mode, uint64_t bin_seed, const uint64_t* bin_keys, int32_t criterion,
                             or_split* out, int32_t* hist_out, int32_t n_threads);

int or_find_splits(const void* x, int dtype, int64_t ld, const int32_t* y, int32_t C,
                   int32_t n_nodes, const int32_t* node_offsets, const int32_t* sample_idx,
                   const int32_t* proj_offsets, const int32_t* nz_offsets,
                   const int32_t* nz_feature, const float* nz_weight,
                   const int32_t* node_bins, int32_t bins, int32_t sort_threshold,
                   int32_t bin_mode, uint64_t bin_seed, int32_t criterion,
                   or_split* out, int32_t* hist_out, int32_t n_threads)
{
    return find_splits_keyed(x, dtype, ld, y, C, n_nodes, node_offsets, sample_idx, proj_offsets, nz_offsets,
                             nz_feature, nz_weight, node_bins, bins, sort_threshold, bin_mode, bin_seed, NULL,
                             criterion, out, hist_out, n_threads);
}

static int find_splits_keyed(const void* x, int dtype, int64_t ld, const int32_t* y, int32_t C,
                             int32_t n_nodes, const int32_t* node_offsets, const int32_t* sample_idx,
                             const int32_t* proj_offsets, const int32_t* nz_offsets,
                             const int32_t* nz_feature, const float* nz_weight,
                             const int32_t* node_bins, int32_t bins, int32_t sort_threshold,
                             int32_t bin_mode, uint64_t bin_seed, const uint64_t* bin_keys, int32_t criterion,
                             or_split* out, int32_t* hist_out, int32_t n_threads)
{
    int32_t P = proj_offsets[n_nodes];
    int T = effective_threshold(sort_threshold);
    cand_t* cands = (cand_t*)calloc((size_t)(P > 0 ? P : 1), sizeof(cand_t));
    int32_t* node_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)(P > 0 ? P : 1));
    int64_t* parent = (int64_t*)calloc((size_t)n_nodes * C + 1, sizeof(int64_t));
    for (int32_t v = 0; v < n_nodes; ++v) {
        for (int32_t q = proj_offsets[v]; q < proj_offsets[v + 1]; ++q)
            node_of[q] = v;
        for (int32_t i = node_offsets[v]; i < node_offsets[v + 1]; ++i)
            parent[(int64_t)v * C + y[sample_idx[i]]] += 1;
    }
    if (hist_out)
        memset(hist_out, 0, sizeof(int32_t) * (size_t)P * bins * C);
#ifdef _OPENMP
    if (n_threads > 0)
        omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int32_t q = 0; q < P; ++q) {
        int32_t v = node_of[q];
        int32_t s0 = node_offsets[v], n = node_offsets[v + 1] - s0;
        int B = node_bins ? node_bins[v] : bins;
        int sort_path = n < T;
        int32_t j0 = nz_offsets[q], z = nz_offsets[q + 1] - j0;
        int32_t* hrow = (hist_out && !sort_path) ? hist_out + (int64_t)q * bins * C : NULL;
        eval_projection(x, dtype, ld, y, C, sample_idx + s0, n, parent + (int64_t)v * C,
                        nz_feature + j0, nz_weight + j0, z, B, sort_path, bin_mode, bin_seed,
                        bin_keys ? (int64_t)bin_keys[q] : (int64_t)q, criterion, &cands[q], hrow, bins);
    }
    for (int32_t v = 0; v < n_nodes; ++v) {
        int32_t n = node_offsets[v + 1] - node_offsets[v];
        int kind = n < T ? 1 : (bin_mode == OR_BINS_RANDOM ? 2 : 0);
        int32_t bestq = -1;
        for (int32_t q = proj_offsets[v]; q < proj_offsets[v + 1]; ++q) {
            if (!cands[q].valid)
                continue;
            if (bestq < 0 ||
                (criterion == OR_CRIT_ENTROPY ? cands[q].E > cands[bestq].E
                                              : q_greater(cands[q].N, cands[q].D, cands[bestq].N, cands[bestq].D)))
                bestq = q;
        }
        if (criterion == OR_CRIT_ENTROPY) {
            if (bestq < 0) {
                no_split(&out[v], kind, n);
                continue;
            }
            const cand_t* b = &cands[bestq];
            double FP = 0.0;
            for (int c = 0; c < C; ++c)
                FP = FP + or_klnk(parent[(int64_t)v * C + c]);
            double ig = ((or_klnk(n) - FP) + b->E) / (double)n;
            if (!(ig > 1e-12)) {
                no_split(&out[v], kind, n);
                continue;
            }
            or_split* o = &out[v];
            memset(o, 0, sizeof(*o));
            o->proj = bestq - proj_offsets[v];
            o->kind = kind;
            o->bin = b->pos;
            o->threshold = b->thr;
            o->lo = b->lo;
            o->scale = b->scale;
            o->n_left = (int32_t)b->nL;
            o->n_right = (int32_t)b->nR;
            o->flags = (b->FL == or_klnk(b->nL) ? 1 : 0) | (b->FR == or_klnk(b->nR) ? 2 : 0);
            o->gain = ig;
            continue;
        }
        uint64_t SP = 0;
        for (int c = 0; c < C; ++c)
            SP += (uint64_t)(parent[(int64_t)v * C + c] * parent[(int64_t)v * C + c]);
        if (bestq < 0) {
            no_split(&out[v], kind, n);
            continue;
        }
        const cand_t* b = &cands[bestq];
        u128 lhs = (u128)(uint64_t)n * b->N;
        u128 rhs = (u128)SP * (u128)b->D;
        if (!(lhs > rhs)) {
            no_split(&out[v], kind, n);
            continue;
        }
        or_split* o = &out[v];
        memset(o, 0, sizeof(*o));
        o->proj = bestq - proj_offsets[v];
        o->kind = kind;
        o->bin = b->pos;
        o->threshold = b->thr;
        o->lo = b->lo;
        o->scale = b->scale;
        o->n_left = (int32_t)b->nL;
        o->n_right = (int32_t)b->nR;
        o->flags = (b->SL == (uint64_t)(b->nL * b->nL) ? 1 : 0) |
                   (b->SR == (uint64_t)(b->nR * b->nR) ? 2 : 0);
        u128 den = (u128)(uint64_t)n * (u128)(uint64_t)n * (u128)b->D;
        o->gain = (double)(lhs - rhs) / (double)den;
    }
    free(parent);
    free(node_of);
    free(cands);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* partition (each node splits its samples between its two children)         */
/* ------------------------------------------------------------------------ */

static int goes_left(const void* x, int dtype, int64_t ld, const int32_t* feat, const float* w,
                     int z, int32_t row, const or_split* s, int B)
{
    float v = or_project_value(x, dtype, ld, feat, w, z, row);
    if (s->kind == 0)
        return or_bin_index(v, s->lo, s->scale, B) <= s->bin;
    if (s->kind == 2)
        return v < s->threshold;   /* random-width: bin(v) <= bin iff v < t_{bin+1} */
    return v <= s->threshold;
}

void or_partition(const void* x, int dtype, int64_t ld, int32_t n_nodes,
                  const int32_t* node_offsets, const int32_t* sample_idx,
                  const int32_t* proj_offsets, const int32_t* nz_offsets,
                  const int32_t* nz_feature, const float* nz_weight,
                  const int32_t* node_bins, int32_t bins, const or_split* splits,
                  int32_t* out_idx, int32_t* child_offsets)
{
    for (int32_t v = 0; v < n_nodes; ++v) {
        int32_t s0 = node_offsets[v], s1 = node_offsets[v + 1];
        const or_split* s = &splits[v];
        child_offsets[2 * v] = s0;
        if (s->proj < 0) {
            for (int32_t i = s0; i < s1; ++i)
                out_idx[i] = sample_idx[i];
            child_offsets[2 * v + 1] = s1;
            continue;
        }
        int32_t q = proj_offsets[v] + s->proj;
        int32_t j0 = nz_offsets[q], z = nz_offsets[q + 1] - j0;
        int B = node_bins ? node_bins[v] : bins;
        int32_t o = s0;
        for (int32_t i = s0; i < s1; ++i)
            if (goes_left(x, dtype, ld, nz_feature + j0, nz_weight + j0, z, sample_idx[i], s, B))
                out_idx[o++] = sample_idx[i];
        child_offsets[2 * v + 1] = o;
        for (int32_t i = s0; i < s1; ++i)
            if (!goes_left(x, dtype, ld, nz_feature + j0, nz_weight + j0, z, sample_idx[i], s, B))
                out_idx[o++] = sample_idx[i];
    }
    child_offsets[2 * n_nodes] = node_offsets[n_nodes];
}

/* ------------------------------------------------------------------------ */
/* projection sampler                                                        */
/* ------------------------------------------------------------------------ */

/* SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014). */
uint64_t or_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* The counter-th output of a SplitMix64 stream started at seed. */
uint64_t or_hash(uint64_t seed, uint64_t counter)
{
    return or_mix64(seed + counter * 0x9E3779B97F4A7C15ULL);
}

uint64_t or_counter(int32_t tree, int32_t level, int32_t pos, int32_t proj, int32_t draw)
{
    uint64_t c = (uint64_t)tree * 64u + (uint64_t)level;
    c = c * (1ull << 24) + (uint64_t)pos;
    c = c * (1ull << 10) + (uint64_t)proj;
    c = c * (1ull << 4) + (uint64_t)draw;
    return c;
}

/* Nonzero count of a projection under the density law (Method: the sparse
 * projection matrix; appendix on Floyd's sampling): each of the d features is
 * kept independently with probability pi = z/d, so the count K follows
 * Binomial(d, pi).  One uniform u in [0, 1) per projection (the top 53 bits
 * of draw 0 of the count stream) replaces the d per-feature coin flips: K is
 * the least k with u < F(k), F the binomial distribution function summed
 * from P(0) = (1 - pi)^d (binary powering, low bit first) with the ratio
 * P(k+1) / P(k) = ((d - k) / (k + 1)) * (pi / (1 - pi)).  K is capped at
 * min(d, 16); if z >= d every feature is kept (then min(d, 16)). */
int32_t or_density_nnz(uint64_t seed, int32_t tree, int32_t level, int32_t pos, int32_t proj, int32_t d,
                       int32_t z)
{
    int32_t cap = d < 16 ? d : 16;
    if (z >= d)
        return cap;
    double pi = (double)z / (double)d;
    double q = 1.0 - pi;
    double ratio = pi / q;
    double p0 = 1.0, b = q;
    for (int32_t e = d; e != 0; e >>= 1) {
        if (e & 1)
            p0 = p0 * b;
        b = b * b;
    }
    uint64_t h = or_hash(seed ^ OR_SEED_NNZ, or_counter(tree, level, pos, proj, 0));
    double u = (double)(h >> 11) / 9007199254740992.0; /* 2^53 */
    double pk = p0, F = p0;
    int32_t k = 0;
    while (k < cap && u >= F) {
        pk = pk * ((double)(d - k) / (double)(k + 1)) * ratio;
        F = F + pk;
        ++k;
    }
    return k;
}

/* Weight of the nonzero of rank s (features ascending).  Signs: bit s of
 * draw 15 (fixed count) or of the weight stream's draw 0 (density law), set
 * = -1.  Uniform: m = top 24 bits of the weight stream's draw s, weight
 * (2m + 1 - 2^24) / 2^24, an odd multiple of 2^-24 in (-1, 1). */
float or_sample_weight(uint64_t seed, int32_t sampler, int32_t weights, int32_t tree, int32_t level,
                       int32_t pos, int32_t proj, int32_t s)
{
    if (weights == OR_WEIGHTS_UNIFORM) {
        uint64_t h = or_hash(seed ^ OR_SEED_WEIGHT, or_counter(tree, level, pos, proj, s));
        int32_t m = (int32_t)(h >> 40);
        return (float)(2 * m + 1 - (1 << 24)) / 16777216.0f;
    }
    uint64_t signs = sampler == OR_SAMPLER_DENSITY
                         ? or_hash(seed ^ OR_SEED_WEIGHT, or_counter(tree, level, pos, proj, 0))
                         : or_hash(seed, or_counter(tree, level, pos, proj, 15));
    return ((signs >> s) & 1u) ? -1.0f : 1.0f;
}

/* One projection: its count nz (z, or the density law above), then nz
 * distinct features out of d by Floyd's algorithm (Bentley and Floyd, "A
 * sample of brilliance", CACM 1987): for j = d-nz .. d-1 draw t uniformly in
 * [0, j]; take t unless already taken, else take j.  The uniform draw is the
 * multiply-shift ((r >> 32) * (j + 1)) >> 32 of draw j - (d - nz).  Features
 * come out ascending with their weights.  Returns nz. */
int32_t or_sample_projection(uint64_t seed, int32_t tree, int32_t level, int32_t pos, int32_t proj,
                             int32_t d, int32_t sampler, int32_t z, int32_t weights, int32_t* feat, float* w)
{
    int32_t nz = sampler == OR_SAMPLER_DENSITY ? or_density_nnz(seed, tree, level, pos, proj, d, z) : z;
    int32_t chosen[16];
    int m = 0;
    for (int32_t j = d - nz; j < d; ++j) {
        uint64_t r = or_hash(seed, or_counter(tree, level, pos, proj, j - (d - nz)));
        int32_t t = (int32_t)(((r >> 32) * (uint64_t)(uint32_t)(j + 1)) >> 32);
        int taken = 0;
        for (int i = 0; i < m; ++i)
            if (chosen[i] == t) taken = 1;
        chosen[m++] = taken ? j : t;
    }
    /* insertion sort ascending */
    for (int i = 1; i < m; ++i) {
        int32_t key = chosen[i];
        int k = i - 1;
        while (k >= 0 && chosen[k] > key) {
            chosen[k + 1] = chosen[k];
            --k;
        }
        chosen[k + 1] = key;
    }
    for (int s2 = 0; s2 < nz; ++s2) {
        feat[s2] = chosen[s2];
        w[s2] = or_sample_weight(seed, sampler, weights, tree, level, pos, proj, s2);
    }
    return nz;
}

/* ------------------------------------------------------------------------ */
/* level-wise growth to purity                                               */
/* ------------------------------------------------------------------------ */

static int32_t majority(const int32_t* y, int C, const int32_t* idx, int32_t n, int* pure)
{
    int64_t cnt[64];
    memset(cnt, 0, sizeof(cnt));
    for (int32_t i = 0; i < n; ++i)
        cnt[y[idx[i]]] += 1;
    int32_t best = 0, nonzero = 0;
    for (int c = 0; c < C; ++c) {
        if (cnt[c] > cnt[best]) best = c;
        if (cnt[c] > 0) nonzero++;
    }
    *pure = nonzero <= 1;
    return best;
}

typedef struct {
    int64_t id;
    int32_t tree;
    int32_t* idx;
    int32_t n;
} fnode_t;

static void init_node(or_tree_node* t, int32_t tree, int32_t depth, int32_t parent, int32_t n,
                      int32_t label)
{
    memset(t, 0, sizeof(*t));
    t->tree = tree;
    t->depth = depth;
    t->parent = parent;
    t->left = -1;
    t->right = -1;
    t->n_samples = n;
    t->label = label;
    t->is_leaf = 1;
    t->kind = -1;
    t->bin = -1;
}

int64_t or_grow_forest(const void* x, int dtype, int64_t ld, int32_t d,
                       const int32_t* y, int32_t C, int32_t n_trees, int32_t first_tree,
                       const int64_t* root_offsets, const int32_t* root_idx,
                       int32_t k, int32_t z, int32_t sampler, int32_t weights, uint64_t seed,
                       int32_t bins, int32_t sort_threshold, int32_t max_depth,
                       int32_t criterion, int32_t bin_mode, uint64_t bin_seed, int32_t n_threads,
                       or_tree_node* nodes, int64_t cap,
                       int64_t* level_nodes, int64_t* level_units)
{
    int64_t n_nodes = 0;
    fnode_t* front = (fnode_t*)malloc(sizeof(fnode_t) * (size_t)(n_trees > 0 ? n_trees : 1));
    int64_t n_front = 0;
    if (cap < n_trees)
        return -1;
    for (int32_t t = 0; t < n_trees; ++t) {
        int32_t n = (int32_t)(root_offsets[t + 1] - root_offsets[t]);
        const int32_t* idx = root_idx + root_offsets[t];
        int pure;
        int32_t label = majority(y, C, idx, n, &pure);
        init_node(&nodes[n_nodes], first_tree + t, 0, -1, n, label);
        if (n >= 2 && !pure && max_depth > 0) {
            nodes[n_nodes].is_leaf = 0;
            front[n_front].id = n_nodes;
            front[n_front].tree = first_tree + t;
            front[n_front].n = n;
            front[n_front].idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
            memcpy(front[n_front].idx, idx, sizeof(int32_t) * (size_t)n);
            n_front++;
        }
        n_nodes++;
    }
    for (int32_t level = 0; n_front > 0; ++level) {
        /* frontier arrays and projections */
        int32_t N = (int32_t)n_front;
        int32_t* off = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N + 1));
        off[0] = 0;
        for (int32_t v = 0; v < N; ++v)
            off[v + 1] = off[v] + front[v].n;
        int32_t* sidx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(off[N] > 0 ? off[N] : 1));
        for (int32_t v = 0; v < N; ++v)
            memcpy(sidx + off[v], front[v].idx, sizeof(int32_t) * (size_t)front[v].n);
        int32_t* po = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N + 1));
        int32_t* no = (int32_t*)malloc(sizeof(int32_t) * ((size_t)N * k + 1));
        int32_t* nf = (int32_t*)malloc(sizeof(int32_t) * ((size_t)N * k * 16 + 1));
        float* nw = (float*)malloc(sizeof(float) * ((size_t)N * k * 16 + 1));
        /* random-width bins of projection p of the node at (tree, level, pos):
         * the sampler's counter without its draw field */
        uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * ((size_t)N * k + 1));
        int32_t pos = 0, tot = 0;
        for (int32_t v = 0; v < N; ++v) {
            if (v > 0 && front[v].tree != front[v - 1].tree)
                pos = 0;
            po[v] = v * k;
            for (int32_t p = 0; p < k; ++p) {
                int64_t q = (int64_t)v * k + p;
                keys[q] = or_counter(front[v].tree, level, pos, p, 0) >> 4;
                no[q] = tot;
                tot += or_sample_projection(seed, front[v].tree, level, pos, p, d, sampler, z, weights, nf + tot,
                                            nw + tot);
            }
            pos++;
        }
        po[N] = N * k;
        no[(int64_t)N * k] = tot;
        if (level_nodes) level_nodes[level] = N;
        if (level_units) level_units[level] = (int64_t)off[N] * k;
        or_split* sp = (or_split*)malloc(sizeof(or_split) * (size_t)N);
        find_splits_keyed(x, dtype, ld, y, C, N, off, sidx, po, no, nf, nw, NULL, bins, sort_threshold, bin_mode,
                          bin_seed, keys, criterion, sp, NULL, n_threads);
        int32_t* pidx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(off[N] > 0 ? off[N] : 1));
        int32_t* coff = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * N + 1));
        or_partition(x, dtype, ld, N, off, sidx, po, no, nf, nw, NULL, bins, sp, pidx, coff);
        fnode_t* next = (fnode_t*)malloc(sizeof(fnode_t) * (size_t)(2 * N));
        int64_t n_next = 0;
        for (int32_t v = 0; v < N; ++v) {
            or_tree_node* me = &nodes[front[v].id];
            if (sp[v].proj < 0) {
                me->is_leaf = 1;
                continue;
            }
            if (n_nodes + 2 > cap) {
                return -1;
            }
            int64_t q = (int64_t)v * k + sp[v].proj;
            me->is_leaf = 0;
            me->kind = sp[v].kind;
            me->bin = sp[v].bin;
            me->threshold = sp[v].threshold;
            me->lo = sp[v].lo;
            me->scale = sp[v].scale;
            me->gain = sp[v].gain;
            me->n_bins = bins;
            me->nnz = no[q + 1] - no[q];
            for (int j = 0; j < me->nnz; ++j) {
                me->feature[j] = nf[no[q] + j];
                me->weight[j] = nw[no[q] + j];
            }
            for (int side = 0; side < 2; ++side) {
                int32_t c0 = coff[2 * v + side];
                int32_t c1 = side == 0 ? coff[2 * v + 1] : off[v + 1];
                int32_t cn = c1 - c0;
                int pure;
                int32_t label = majority(y, C, pidx + c0, cn, &pure);
                int64_t cid = n_nodes++;
                init_node(&nodes[cid], front[v].tree, level + 1, (int32_t)front[v].id, cn, label);
                if (side == 0) me->left = (int32_t)cid;
                else me->right = (int32_t)cid;
                if (cn >= 2 && !pure && level + 1 < max_depth) {
                    nodes[cid].is_leaf = 0;
                    next[n_next].id = cid;
                    next[n_next].tree = front[v].tree;
                    next[n_next].n = cn;
                    next[n_next].idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)cn);
                    memcpy(next[n_next].idx, pidx + c0, sizeof(int32_t) * (size_t)cn);
                    n_next++;
                }
            }
        }
        for (int64_t v = 0; v < n_front; ++v)
            free(front[v].idx);
        free(front);
        front = next;
        n_front = n_next;
        free(off); free(sidx); free(po); free(no); free(nf); free(nw); free(keys); free(sp); free(pidx); free(coff);
    }
    free(front);
    return n_nodes;
}

/* ------------------------------------------------------------------------ */
/* prediction (the forest's trees each vote the label of the leaf a row      */
/* reaches; the majority class wins, ties to the lowest class)               */
/* ------------------------------------------------------------------------ */

static int node_goes_left(const void* x, int dtype, int64_t ld, const or_tree_node* t, int32_t row)
{
    float v = or_project_value(x, dtype, ld, t->feature, t->weight, t->nnz, row);
    if (t->kind == 0)
        return or_bin_index(v, t->lo, t->scale, t->n_bins) <= t->bin;
    if (t->kind == 2)
        return v < t->threshold;
    return v <= t->threshold;
}

int32_t or_leaf_of(const void* x, int dtype, int64_t ld, const or_tree_node* nodes, int32_t root,
                   int32_t row)
{
    int32_t i = root;
    while (!nodes[i].is_leaf)
        i = node_goes_left(x, dtype, ld, &nodes[i], row) ? nodes[i].left : nodes[i].right;
    return i;
}

void or_predict(const void* x, int dtype, int64_t ld, const or_tree_node* nodes, const int32_t* roots,
                int32_t n_trees, int32_t C, int32_t n_rows, int32_t* votes, int32_t* pred)
{
    for (int32_t r = 0; r < n_rows; ++r) {
        int32_t* vr = votes + (int64_t)r * C;
        for (int c = 0; c < C; ++c)
            vr[c] = 0;
        for (int32_t t = 0; t < n_trees; ++t)
            vr[nodes[or_leaf_of(x, dtype, ld, nodes, roots[t], r)].label] += 1;
        int32_t best = 0;
        for (int c = 1; c < C; ++c)
            if (vr[c] > vr[best])
                best = c;
        pred[r] = best;
    }
}
