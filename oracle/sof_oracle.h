/*
 * sof_oracle.h -- reference CPU implementation of per-node split search for
 * sparse oblique forests.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this code.  The GPU library never calls,
 * links or includes it, and it shares no source with the GPU library.
 *
 * Method (paper section 4, "Method", steps 1-3, and section 4.1, dynamic
 * histogramming): for every node of a frontier and every one of its sparse
 * projections, (1) form the projected value of each active sample as a +/-1
 * weighted sum of a few feature columns, (2) either count per-class samples in
 * equal-width bins over the node's [min, max] or sort the projected values when
 * the node is small, (3) scan the boundaries for the best split criterion and
 * keep the best over projections.  The criterion is Gini impurity decrease
 * (the paper's YDF uses entropy; this build fixes Gini).
 *
 * Arithmetic is plain IEEE binary32 for projections and binning (compiled with
 * -ffp-contract=off), exact integers for counts and for comparing candidates,
 * and binary64 only for the reported gain.
 */
#ifndef SOF_ORACLE_H
#define SOF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_F32 0
#define OR_F16 1

/* Nodes with at most this many samples can take the sort path; a sort
 * threshold above OR_SORT_LIMIT + 1 acts as OR_SORT_LIMIT + 1. */
#define OR_SORT_LIMIT 8192

/* Split criteria. */
#define OR_CRIT_GINI    0
#define OR_CRIT_ENTROPY 1

/* Bin layouts of the histogram path. */
#define OR_BINS_EQUAL  0
#define OR_BINS_RANDOM 1

/* projection sampler of growth: nonzero-count law and weight law */
#define OR_SAMPLER_FIXED   0
#define OR_SAMPLER_DENSITY 1
#define OR_WEIGHTS_SIGN    0
#define OR_WEIGHTS_UNIFORM 1
#define OR_SEED_NNZ    0x6A09E667F3BCC909ULL
#define OR_SEED_WEIGHT 0xBB67AE8584CAA73BULL

typedef struct {
    int32_t proj;      /* node-local index of the winning projection, -1 = no split */
    int32_t kind;      /* 0 = histogram path (equal width), 1 = sort path, 2 = histogram path
                          (random width); the node's path even without a split */
    int32_t bin;       /* hist: left iff bin(v) <= bin; sort: sorted position, left = first bin+1 */
    float   threshold; /* sort: left iff v <= threshold; random width: left iff v < threshold
                          (= boundary bin+1); equal width: lo + (bin+1)/scale (informational) */
    float   lo;        /* minimum projected value of the winning projection */
    float   scale;     /* hist: B / (hi - lo) with the overflow guard; sort: 0 */
    int32_t n_left, n_right;
    int32_t flags;     /* bit 0: left child pure, bit 1: right child pure */
    int32_t pad;
    double  gain;      /* Gini(parent) - weighted Gini(children); exactly 0 without a split */
} or_split;

typedef struct {
    int32_t tree, depth, parent, left, right;
    int32_t n_samples, label, is_leaf;
    int32_t kind, bin;
    float   threshold, lo, scale;
    int32_t n_bins, nnz, pad;
    int32_t feature[16];
    float   weight[16];
    double  gain;
} or_tree_node;

/* IEEE binary16 -> binary32 (exact). */
float or_half_to_float(uint16_t h);

/* Projected value of one row for one projection (CSR order, from +0.0f). */
float or_project_value(const void* x, int dtype, int64_t ld, const int32_t* feat,
                       const float* w, int z, int32_t row);

/* Equal-width bin parameters and bin index (see the header of the .c file). */
float or_bin_scale(int n_bins, float lo, float hi);
int   or_bin_index(float v, float lo, float scale, int n_bins);

/* Random-width boundaries t[0..n_bins-2] of projection q, and the bin of v
 * (the number of boundaries <= v). */
void or_rw_boundaries(uint64_t seed, int64_t q, int n_bins, float lo, float hi, float* t);
int  or_rw_bin(const float* t, int n_bins, float v);

/* Projected values of every (node, projection, sample), node blocks in node
 * order, each block laid out [projection][sample]. */
void or_project(const void* x, int dtype, int64_t ld, int32_t n_nodes,
                const int32_t* node_offsets, const int32_t* sample_idx,
                const int32_t* proj_offsets, const int32_t* nz_offsets,
                const int32_t* nz_feature, const float* nz_weight, float* out);

/* Best split of every frontier node.  hist_out (optional) receives
 * [projection][bins][n_classes] int32 counts for histogram-path nodes and zeros
 * elsewhere (bins = the maximum bin count, entries b >= B_v are zero). */
int or_find_splits(const void* x, int dtype, int64_t ld, const int32_t* y, int32_t n_classes,
                   int32_t n_nodes, const int32_t* node_offsets, const int32_t* sample_idx,
                   const int32_t* proj_offsets, const int32_t* nz_offsets,
                   const int32_t* nz_feature, const float* nz_weight,
                   const int32_t* node_bins, int32_t bins, int32_t sort_threshold,
                   int32_t bin_mode, uint64_t bin_seed, int32_t criterion,
                   or_split* out, int32_t* hist_out, int32_t n_threads);

/* Natural logarithm of an integer k >= 1 by a fixed sequence of IEEE binary64
 * operations, and f(k) = k ln k (the entropy criterion's building block). */
double or_ln_int(int64_t k);
double or_klnk(int64_t k);

/* Stable partition of every node's samples by its split: left block (input
 * order) then right block (input order).  child_offsets has 2N+1 entries. */
void or_partition(const void* x, int dtype, int64_t ld, int32_t n_nodes,
                  const int32_t* node_offsets, const int32_t* sample_idx,
                  const int32_t* proj_offsets, const int32_t* nz_offsets,
                  const int32_t* nz_feature, const float* nz_weight,
                  const int32_t* node_bins, int32_t bins, const or_split* splits,
                  int32_t* out_idx, int32_t* child_offsets);

/* Counter-based projection sampler. */
uint64_t or_mix64(uint64_t z);
uint64_t or_hash(uint64_t seed, uint64_t counter);
uint64_t or_counter(int32_t tree, int32_t level, int32_t pos, int32_t proj, int32_t draw);
int32_t or_density_nnz(uint64_t seed, int32_t tree, int32_t level, int32_t pos, int32_t proj,
                       int32_t n_features, int32_t z);
float or_sample_weight(uint64_t seed, int32_t sampler, int32_t weights, int32_t tree, int32_t level,
                       int32_t pos, int32_t proj, int32_t rank);
int32_t or_sample_projection(uint64_t seed, int32_t tree, int32_t level, int32_t pos, int32_t proj,
                             int32_t n_features, int32_t sampler, int32_t z, int32_t weights,
                             int32_t* feat, float* w);

/* Level-wise growth of several trees to purity (tree ids first_tree ..
 * first_tree + n_trees - 1 key the sampler).  Returns the number of nodes,
 * or -1 if cap is too small.  level_nodes / level_units (optional, length
 * max_depth + 1) receive the frontier size and sum n_v*k per level.  With
 * random-width bins, projection p of the node at (tree, level, pos) takes the
 * width stream key or_counter(tree, level, pos, p, 0) >> 4 in place of its
 * index in the level's call. */
int64_t or_grow_forest(const void* x, int dtype, int64_t ld, int32_t n_features,
                       const int32_t* y, int32_t n_classes, int32_t n_trees, int32_t first_tree,
                       const int64_t* root_offsets, const int32_t* root_idx,
                       int32_t k, int32_t z, int32_t sampler, int32_t weights, uint64_t seed,
                       int32_t bins,
                       int32_t sort_threshold, int32_t max_depth,
                       int32_t criterion, int32_t bin_mode, uint64_t bin_seed, int32_t n_threads,
                       or_tree_node* nodes, int64_t cap,
                       int64_t* level_nodes, int64_t* level_units);

/* Leaf a row reaches from a root, and forest prediction: per row, every tree
 * votes its leaf's label; pred = the class with most votes (lowest on ties).
 * Internal nodes send a row left when bin(v) <= bin (kind 0), v <= threshold
 * (kind 1) or v < threshold (kind 2), v being the node's projection. */
int32_t or_leaf_of(const void* x, int dtype, int64_t ld, const or_tree_node* nodes, int32_t root,
                   int32_t row);
void or_predict(const void* x, int dtype, int64_t ld, const or_tree_node* nodes, const int32_t* roots,
                int32_t n_trees, int32_t n_classes, int32_t n_rows, int32_t* votes, int32_t* pred);

#ifdef __cplusplus
}
#endif

#endif
