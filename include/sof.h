/*
 * sof.h -- split search for sparse oblique forests on AMD Instinct MI355X
 * (gfx950).  C ABI: plain pointers and sizes, no C++ or framework types.
 *
 * The method is the per-node split search of "Vectorized Adaptive Histograms
 * for Sparse Oblique Forests" (section 4, steps 1-3; section 4.1 for the
 * switch between histograms and sorting; section 4.3 for the data resident on
 * the device and a call that returns the best projection and its split).  For
 * every node of a frontier and each of its sparse projections the library
 *   1. forms the projected value of every active sample, a weighted sum of a
 *      few feature columns (+/-1, integer or FP32 weights) accumulated in FP32
 *      in CSR order from +0.0f;
 *   2. builds per-class counts over equal-width (or random-width) bins
 *      spanning the node's [min, max] of that projection (histogram path), or
 *      sorts the projected values when the node has fewer than the sort
 *      threshold samples;
 *   3. scans the bin (or sorted-sample) boundaries for the largest Gini
 *      impurity decrease, compared exactly in integers (or the largest
 *      information gain, SOF_CRIT_ENTROPY), and keeps the best over
 *      projections (ties: lowest projection, then lowest bin or position);
 * and then stably partitions each node's sample indices between its children.
 * Forests grow level by level on the device (sof_grow_level), drawing their
 * projections with a counter-based sampler, and predict (sof_predict).
 *
 * Conventions shared by every call:
 *  - Array pointers inside sof_data / sof_frontier / sof_proj / sof_params and
 *    every output pointer are DEVICE pointers owned by the caller; the library
 *    never frees caller memory.  Host-side counts in those structs must match
 *    the device arrays (checked on the device only when SOF_CHECK=1 is set in
 *    the environment; otherwise a mismatch is undefined behaviour).
 *  - Compute calls are asynchronous on `stream` (a hipStream_t passed as void*,
 *    NULL = the default stream), allocate nothing and do not synchronise; they
 *    can be captured in a HIP graph.  sof_create, sof_forest_create,
 *    sof_forest_frontier_size, sof_forest_frontier_stats, sof_forest_export
 *    and sof_autotune allocate
 *    and/or synchronise.
 *  - Every call returns a status; sof_last_error() gives a thread-local message
 *    for the last failure.  Host-side argument checks run before any launch
 *    and need no GPU.
 *
 * Data layout:
 *  - features: x[f * ld + r] for feature f < n_features and row r < n_rows
 *    (column store: each feature contiguous), FP32 or FP16;
 *  - labels: int32 y[r] in [0, n_classes);
 *  - frontier: node v owns sample_idx[node_offsets[v] .. node_offsets[v+1]);
 *  - projections (CSR): node v owns projections proj_offsets[v] ..
 *    proj_offsets[v+1]; projection q owns nonzeros nz_offsets[q] ..
 *    nz_offsets[q+1] with feature ids nz_feature[] (distinct within a
 *    projection) and weights nz_weight[] in {-1, +1}.
 */
#ifndef SOF_H
#define SOF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SOF_OK               0
#define SOF_ERR_INVALID_ARG (-1)  /* a null pointer, a size out of range, inconsistent counts */
#define SOF_ERR_UNSUPPORTED (-2)  /* dtype, class count, bin count or device not supported */
#define SOF_ERR_WORKSPACE   (-3)  /* workspace missing, too small or misaligned */
#define SOF_ERR_OVERFLOW    (-4)  /* a node above 2^24 samples, totals above 2^31-1 */
#define SOF_ERR_HIP         (-5)  /* a HIP runtime call failed; the message names it */
#define SOF_ERR_DEVICE      (-6)  /* a device-side content check failed (SOF_CHECK=1) */

/* feature storage types */
#define SOF_F32 0
#define SOF_F16 1

/* limits */
#define SOF_MAX_BINS         256
#define SOF_MIN_BINS         2
#define SOF_MAX_CLASSES      16
#define SOF_MAX_NNZ          16          /* nonzeros per projection */
#define SOF_MAX_NODE_SAMPLES (1 << 24)   /* exact 128-bit comparisons need n <= 2^24 */
#define SOF_SORT_LIMIT       8192        /* largest node that can take the sort path */
#define SOF_WORKSPACE_ALIGN  256
#define SOF_STATIC_SCRATCH_BYTES (64 << 20)  /* per-device scratch of sof_find_splits_noalloc */

/* split kinds */
#define SOF_SPLIT_HIST  0   /* histogram path, equal-width bins */
#define SOF_SPLIT_SORT  1   /* sort path */
#define SOF_SPLIT_RHIST 2   /* histogram path, random-width bins */

/* split criteria (sof_params.criterion) */
#define SOF_CRIT_GINI    0
#define SOF_CRIT_ENTROPY 1

/* bin layouts of the histogram path (sof_params.bin_mode) */
#define SOF_BINS_EQUAL  0
#define SOF_BINS_RANDOM 1

/* Projection sampler of tree growth (sof_forest_desc.sampler, .weights). */
#define SOF_SAMPLER_FIXED   0   /* exactly z distinct features per projection */
#define SOF_SAMPLER_DENSITY 1   /* each feature with probability z/d: Binomial(d, z/d) of them */
#define SOF_WEIGHTS_SIGN    0   /* weights +1 / -1 */
#define SOF_WEIGHTS_UNIFORM 1   /* weights uniform on (-1, 1), never 0, exact in FP32 */

typedef struct sof_ctx sof_ctx;
typedef struct sof_forest sof_forest;

typedef struct {
    const void*    x;           /* device, x[f * ld + r] */
    const int32_t* y;           /* device, n_rows labels */
    int64_t        ld;          /* >= n_rows */
    int32_t        n_rows;
    int32_t        n_features;
    int32_t        n_classes;   /* 2..SOF_MAX_CLASSES */
    int32_t        dtype;       /* SOF_F32 or SOF_F16 */
} sof_data;

typedef struct {
    const int32_t* node_offsets;  /* device, n_nodes + 1, non-decreasing, [0] = 0 */
    const int32_t* sample_idx;    /* device, n_samples row ids (repeats allowed) */
    int64_t        n_samples;     /* = node_offsets[n_nodes] */
    int32_t        n_nodes;
    int32_t        max_node_samples; /* >= every node's sample count (host-known bound) */
} sof_frontier;

typedef struct {
    const int32_t* proj_offsets;  /* device, n_nodes + 1 */
    const int32_t* nz_offsets;    /* device, n_proj + 1 */
    const int32_t* nz_feature;    /* device, n_nz */
    const int8_t*  nz_weight;     /* device, n_nz integer weights (usually -1 or +1); not read
                                     when nz_value is given */
    int64_t        n_nz;          /* = nz_offsets[n_proj] */
    int32_t        n_proj;        /* = proj_offsets[n_nodes] */
    int32_t        max_proj_per_node; /* >= every node's projection count, <= 1024 */
    const float*   nz_value;      /* device, n_nz finite FP32 weights, or NULL (then nz_weight) */
} sof_proj;

/* Projected value of a sample (Method, step 1): v = sum over the projection's
 * nonzeros in CSR order of w_j * x[f_j][row], each product and each add one
 * FP32 rounding (no fused multiply-add), starting from +0.  With weights
 * +/-1 every product is exact. */

/* Histogram bins.  SOF_BINS_EQUAL: B equal-width bins over [lo, hi] (the
 * Method section's "few arithmetic operations" binning).  SOF_BINS_RANDOM:
 * boundaries at random-width intervals (the Introduction's footnote; the
 * paper gives no sampling rule, so this one is the library's): for the q-th
 * projection of the call (q = proj_offsets[v] + p) the bin widths are
 * g_j = 1 + (bits 63..48 of SplitMix64 output 256 q + j of the stream started
 * at bin_seed), j = 0..B-1; with G_i = g_0 + ... + g_{i-1}, boundary i
 * (i = 1..B-1) is lo + (G_i / G_B) * (hi - lo), each operation one FP32
 * rounding, and a value's bin is the number of boundaries <= v. */
typedef struct {
    const int32_t* node_bins;     /* device, n_nodes bin counts in [2, bins], or NULL */
    int32_t        bins;          /* 2..SOF_MAX_BINS: bin count when node_bins is NULL, else the maximum */
    int32_t        sort_threshold;/* nodes with n < min(T, SOF_SORT_LIMIT + 1) sort; 0 = all histogram */
    int32_t        bin_mode;      /* SOF_BINS_EQUAL or SOF_BINS_RANDOM */
    int32_t        criterion;     /* SOF_CRIT_GINI or SOF_CRIT_ENTROPY, on both paths */
    uint64_t       bin_seed;      /* SOF_BINS_RANDOM: seed of the widths */
    /* Wave tile of the histogram path (the results do not depend on it):
     * nodes of up to small_max samples take one wave per projection, larger
     * ones up to mid_split one block per 4 projections with up to 16 samples
     * per thread, larger ones up to 8192 the same with 32 per thread.
     * small_max in [256, 512], mid_split in [2048, 4096]; 0 picks 512 and
     * 4096 (sof_autotune measures both choices). */
    int32_t        small_max;
    int32_t        mid_split;
} sof_params;

/* Criteria.  SOF_CRIT_GINI: Gini decrease, argmax by exact 128-bit integer
 * comparisons.  SOF_CRIT_ENTROPY (information gain, YDF's criterion in the
 * Method section): each boundary's E = sum_c f(l_c) + sum_c f(r_c) - f(n_L)
 * - f(n_R), f(k) = k ln k, in binary64 with a natural log built from IEEE
 * basic operations (reduction to [sqrt(2)/2, sqrt(2)), 12 atanh-series terms),
 * the sums over classes ascending, at every bin boundary (histogram path) or
 * every boundary between distinct sorted values (sort path); the largest E
 * wins (lowest projection, then bin or sorted position, on ties), the gain
 * is ((f(n) - sum_c f(P_c)) + E) / n and the node splits iff it exceeds
 * 1e-12. */

/* Best split of one node (section 4.3: the projection and its split value). */
typedef struct {
    int32_t proj;       /* node-local index of the winning projection, -1 = no split */
    int32_t kind;       /* SOF_SPLIT_HIST, _SORT or _RHIST: the node's path (also without a split) */
    int32_t bin;        /* hist: left iff bin(v) <= bin; sort: sorted position, left = first bin+1; -1 */
    float   threshold;  /* sort: left iff v <= threshold; random-width hist: left iff v < threshold
                           (boundary bin+1); equal-width hist: lo + (bin+1)/scale, informational */
    float   lo;         /* min projected value of the winner */
    float   scale;      /* hist: bins / (hi - lo), FLT_MAX if that is not finite; sort: 0 */
    int32_t n_left;     /* no split: n_left = n, n_right = 0 */
    int32_t n_right;
    int32_t flags;      /* bit 0: left child pure, bit 1: right child pure */
    float   gain;       /* Gini(parent) - weighted Gini(children) in FP32; 0 without a split */
} sof_split;

/* Node of an exported tree.  Ids are positions in the forest's creation
 * order: roots first, then level by level, children in frontier order, left
 * before right. */
typedef struct {
    int32_t tree, depth, parent, left, right;   /* -1 where absent */
    int32_t n_samples, label, is_leaf;          /* label: majority class, lowest id on ties */
    int32_t kind, bin;                          /* split rule (kind -1 for leaves) */
    float   threshold, lo, scale;
    int32_t n_bins, nnz, pad;
    int32_t feature[16];                        /* the winning projection: nnz features, ascending */
    float   weight[16];                         /* ... and their weights (0 past nnz) */
    double  gain;
} sof_tree_node;

typedef struct {
    const int64_t* root_offsets;  /* HOST, n_trees + 1: tree t owns root_idx[root_offsets[t] ..) */
    const int32_t* root_idx;      /* device, root sample ids of every tree (e.g. a bootstrap) */
    uint64_t       seed;          /* projection sampler seed */
    int32_t        n_trees;
    int32_t        first_tree;    /* tree ids first_tree .. first_tree+n_trees-1 key the sampler */
    int32_t        k;             /* projections per node, 1..1024 */
    int32_t        z;             /* SOF_SAMPLER_FIXED: nonzeros per projection, 1..15, <= n_features;
                                     SOF_SAMPLER_DENSITY: their mean, 1..16 (density z / n_features) */
    int32_t        bins;          /* 2..256 */
    int32_t        sort_threshold;
    int32_t        max_depth;     /* 0..64: nodes at this depth become leaves */
    int32_t        sampler;       /* SOF_SAMPLER_FIXED or SOF_SAMPLER_DENSITY */
    int32_t        weights;       /* SOF_WEIGHTS_SIGN or SOF_WEIGHTS_UNIFORM */
    int32_t        criterion;     /* SOF_CRIT_GINI or SOF_CRIT_ENTROPY */
    int32_t        bin_mode;      /* SOF_BINS_EQUAL or SOF_BINS_RANDOM */
    int32_t        pad;
    uint64_t       bin_seed;      /* SOF_BINS_RANDOM: seed of the widths; projection p of the node at
                                     (tree, level, pos) takes the width stream index
                                     ((tree * 64 + level) << 24 + pos) << 10 + p in place of the
                                     projection's index in the call */
} sof_forest_desc;

/* The sampler (Method: the sparse projection matrix; appendix: Floyd's
 * sampling).  Projection p of node (tree, level, pos) depends on those values
 * and the seed only; each random number is the SplitMix64 output at counter
 * ((((tree * 64 + level) << 24 + pos) << 10 + p) << 4) + draw of a stream
 * started at seed, seed ^ 0x6A09E667F3BCC909 (the nonzero count) or
 * seed ^ 0xBB67AE8584CAA73B (weights).
 *   nonzero count: FIXED: z.  DENSITY: pi = z/d, q = 1 - pi, r = pi/q,
 *     P(0) = q^d by binary powering (low bit first), P(k+1) = (P(k) *
 *     ((d-k)/(k+1))) * r; the count is the least k with
 *     u < P(0) + ... + P(k), u = (output >> 11) / 2^53, at most min(d, 16);
 *     each operation one binary64 rounding.  (d if z >= d, at most 16.)
 *   features: Floyd's algorithm, draw j = 0..z_p-1 proposes
 *     t = ((output >> 32) * (d - z_p + j + 1)) >> 32 and takes d - z_p + j if
 *     t is taken; stored ascending.
 *   weights of the nonzero of rank s: SIGN: -1 iff bit s of draw 15 (FIXED)
 *     or of the weight stream's draw 0 (DENSITY) is set; UNIFORM:
 *     (2m + 1 - 2^24) / 2^24, m = weight-stream draw s >> 40. */

typedef struct {
    int32_t sort_threshold;   /* chosen histogram/sort switch T */
    int32_t bins_small;       /* bin count for nodes below bins_switch */
    int32_t bins_switch;      /* nodes with n < bins_switch use bins_small, others the caller's bins */
    int32_t n_points;         /* measured sizes */
    float   sort_us[32];      /* per measured size: sort-path time per node-projection (us) */
    float   hist_us[32];      /* per measured size: histogram-path time per node-projection (us) */
    int32_t sizes[32];
    float   elapsed_ms;       /* wall time of the whole tuning run */
    float   half_us[32];      /* per measured size: histogram path with bins_small bins (us) */
    int32_t small_max;        /* chosen wave tile (sof_params.small_max, mid_split) */
    int32_t mid_split;
    /* per measured size in 257..512 (2049..4096), on a frontier of at least 4
     * nodes per compute unit: the histogram path with the default tile and
     * with the block tile (32 samples per thread) (us); 0 elsewhere.  An edge
     * moves below a size when the other tile is more than 5% faster there
     * and at every larger size of its range. */
    float   tile_base_us[32];
    float   tile_us[32];
} sof_tune;

/* ---------------------------------------------------------------------- */

/* Library version string (static storage). */
const char* sof_version(void);

/* Message for the last failed call on this thread ("" if none). */
const char* sof_last_error(void);

/* Create a context on HIP device `device`: checks the architecture (gfx950),
 * sizes the persistent launches from the device's compute-unit count and
 * occupancy, creates the two auxiliary streams (default priority) and three
 * events that the batched search forks its size classes onto, and takes the
 * device address of the static scratch of sof_find_splits_noalloc.  Allocates
 * no device memory.  Errors: SOF_ERR_INVALID_ARG (null
 * out), SOF_ERR_HIP, SOF_ERR_UNSUPPORTED (not gfx950). */
int sof_create(int device, sof_ctx** out);
int sof_destroy(sof_ctx* ctx);

/* Bytes of device workspace that sof_project, sof_find_splits and
 * sof_partition need for these sizes (the maximum over the three).  Pure host
 * arithmetic; runs without a GPU when ctx is NULL.  Errors as the calls. */
int sof_workspace_size(const sof_ctx* ctx, const sof_data* data, const sof_frontier* frontier,
                       const sof_proj* proj, const sof_params* params, size_t* bytes);

/* Step 1 alone (section 4, step 1): projected values of every (node,
 * projection, sample), node blocks in node order, each block [projection]
 * [sample] in frontier sample order.  out has sum_v k_v * n_v floats.
 * ws: device workspace of at least sof_workspace_size bytes, 256-byte aligned. */
int sof_project(sof_ctx* ctx, const sof_data* data, const sof_frontier* frontier,
                const sof_proj* proj, float* out, void* ws, size_t ws_bytes, void* stream);

/* Steps 1-3 for a whole frontier in one batched launch sequence: writes the
 * best split of every node to out[n_nodes].  hist_out (optional, NULL to skip)
 * receives int32 counts [n_proj][params->bins][n_classes] for histogram-path
 * nodes (entries beyond a node's bin count and all entries of sort-path nodes
 * are zero).  Errors: SOF_ERR_INVALID_ARG, SOF_ERR_UNSUPPORTED,
 * SOF_ERR_WORKSPACE, SOF_ERR_OVERFLOW, SOF_ERR_HIP. */
int sof_find_splits(sof_ctx* ctx, const sof_data* data, const sof_frontier* frontier,
                    const sof_proj* proj, const sof_params* params, sof_split* out,
                    int32_t* hist_out, void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): sof_find_splits
 * with its workspace in a static per-device array of SOF_STATIC_SCRATCH_BYTES
 * (64 MiB, allocated with the library's code object on every device it runs
 * on and held until the process ends; its address is taken by sof_create).
 * Same arguments, outputs and errors as sof_find_splits, without ws; calls
 * no hipMalloc, hipFree or allocating routine.  Differences: big nodes
 * (above 8192 samples) re-gather their columns instead of caching projected
 * values, SOF_CHECK content checks are skipped, and sizes whose workspace
 * exceeds the array fail with SOF_ERR_WORKSPACE before any launch.  Every
 * call on a device uses the same array, so calls that overlap in time on
 * one device (two streams, two threads) race and must be serialised by the
 * caller; a call needs no clearing from the previous one. */
int sof_find_splits_noalloc(sof_ctx* ctx, const sof_data* data, const sof_frontier* frontier,
                            const sof_proj* proj, const sof_params* params, sof_split* out,
                            int32_t* hist_out, void* stream);

/* Stable partition (section 4: each node splits its samples between its
 * children): out_idx (same size as sample_idx, must not alias it) receives,
 * per node, the samples going left in input order then those going right in
 * input order, re-evaluating the split rule on recomputed projected values.
 * child_offsets[2N+1]: [2v] = node start, [2v+1] = start of the right block,
 * [2N] = n_samples.  A node without a split keeps all samples on the left.
 * The left count is measured, not taken from splits[v].n_left. */
int sof_partition(sof_ctx* ctx, const sof_data* data, const sof_frontier* frontier,
                  const sof_proj* proj, const sof_params* params, const sof_split* splits,
                  int32_t* out_idx, int32_t* child_offsets, void* ws, size_t ws_bytes,
                  void* stream);

/* Forest growth to purity, level by level (sections 2 and 4.1: trees trained
 * to purity; section 6: several nodes and trees batched into single launches).
 * sof_forest_create allocates the forest's device state (frontier buffers,
 * node table, workspace) for the trees in desc; data must stay valid. */
int sof_forest_create(sof_ctx* ctx, const sof_data* data, const sof_forest_desc* desc,
                      sof_forest** out);
int sof_forest_destroy(sof_forest* forest);

/* One level for every tree: sample k projections per frontier node on the
 * device (counter-based SplitMix64 hash, Floyd's distinct sampling), find the
 * splits, partition, record nodes and build the next frontier.  Asynchronous;
 * replays a captured HIP graph per level when use_graph is nonzero. */
int sof_grow_level(sof_forest* forest, int use_graph, void* stream);

/* Nodes in the current frontier (0 = the forest is complete).  Synchronises
 * the stream (one 4-byte device-to-host copy). */
int sof_forest_frontier_size(sof_forest* forest, int64_t* n_nodes, void* stream);

/* The current frontier of the forest: its node count, the total samples of
 * those nodes (the projection units of the next level are n_samples * k) and
 * the depth of its nodes.  Synchronises the stream (one 32-byte
 * device-to-host copy).  Errors: SOF_ERR_INVALID_ARG (NULL), SOF_ERR_HIP. */
int sof_forest_frontier_stats(sof_forest* forest, int64_t* n_nodes, int64_t* n_samples, int32_t* depth,
                              void* stream);

/* Copy the node table to host memory (synchronises).  *n receives the node
 * count; SOF_ERR_INVALID_ARG when cap is smaller. */
int sof_forest_export(sof_forest* forest, sof_tree_node* host_nodes, int64_t cap, int64_t* n,
                      void* stream);

/* Forest prediction (the trees of section 2 vote): for every row r < n_rows
 * of data (labels unused, may be NULL), walk each tree from its root node;
 * an internal node sends the row left when its rule holds on the row's
 * projection v (the node's features and +/-1 weights, FP32 adds in order
 * from +0): kind SOF_SPLIT_HIST bin(v) <= bin with the node's lo, scale and
 * n_bins; SOF_SPLIT_SORT v <= threshold; SOF_SPLIT_RHIST v < threshold.  The
 * leaf's label gets one vote.  nodes: device array of n_nodes records in
 * sof_forest_export's layout (8-byte aligned); roots: device array of n_trees
 * root indices (a forest's roots are nodes 0 .. n_trees-1); votes (optional,
 * device, n_rows * n_classes int32) and pred (device, n_rows int32: the class
 * with most votes, the lowest on ties).  A child index outside [0, n_nodes)
 * ends the walk without a vote.  Asynchronous on stream; allocates nothing.
 * Errors: SOF_ERR_INVALID_ARG, SOF_ERR_UNSUPPORTED (dtype, classes),
 * SOF_ERR_HIP. */
int sof_predict(sof_ctx* ctx, const sof_data* data, const sof_tree_node* nodes, int64_t n_nodes,
                const int32_t* roots, int32_t n_trees, int32_t* votes, int32_t* pred, void* stream);

/* Crossover microbenchmark (section 4.1: run once before training, a search
 * for the node size where histograms overtake sorting): times the sort and
 * histogram paths on synthetic frontiers (2^16 rows) of equal nodes of
 * growing size (2 .. 8192), on this device, with the caller's storage type
 * (SOF_F32 or SOF_F16), class count, projections per node (capped at 64 for
 * timing), nonzeros per projection and bin count.  Picks the sort threshold
 * (the smallest measured size from which the histogram path is never slower;
 * sizes above two consecutive histogram wins are not sorted, their sort_us is
 * 0) and a bin-count switch for small nodes (half the bins below the smallest
 * measured size from which full bins cost at most 10% more than half bins at
 * every larger size, half bins being timed up to 1024 samples; 0 when that
 * holds everywhere).  Allocates its own device buffers, frees
 * them, and synchronises `stream`.  Errors: SOF_ERR_INVALID_ARG (NULL, k or
 * nnz out of range), SOF_ERR_UNSUPPORTED (dtype, classes, bins), SOF_ERR_HIP. */
int sof_autotune(sof_ctx* ctx, int32_t dtype, int32_t n_classes, int32_t k, int32_t nnz, int32_t bins,
                 sof_tune* out, void* stream);

/* The same microbenchmark on the caller's own data: the frontiers take rows
 * 0 .. min(n_rows, 2^16) - 1 of data (its labels and its first min(d, 64)
 * features, its storage type and class count), so the crossover reflects the
 * caller's value distribution.  data must stay valid during the call.
 * Errors: as sof_autotune, and SOF_ERR_INVALID_ARG when data has fewer
 * features than nnz. */
int sof_autotune_on(sof_ctx* ctx, const sof_data* data, int32_t k, int32_t nnz, int32_t bins,
                    sof_tune* out, void* stream);

/* Benchmark instrumentation.  The launch sequence of sof_find_splits runs in
 * these stages, in this order: */
enum {
    SOF_STAGE_PLAN = 0,   /* counter reset, node classification, queue expansion */
    SOF_STAGE_BIG_RANGE,  /* nodes above 8192 samples: range of each (projection, chunk) */
    SOF_STAGE_BIG_MERGE,  /* ... range of each projection over the node */
    SOF_STAGE_BIG_HIST,   /* ... class histogram of each (projection, chunk) */
    SOF_STAGE_BIG_SCAN,   /* ... summed histograms, boundary scan */
    SOF_STAGE_MID,        /* histogram nodes of 513..4096 samples */
    SOF_STAGE_MID2,       /* histogram nodes of 4097..8192 samples */
    SOF_STAGE_SMALL,      /* histogram nodes up to 512, sort nodes up to 64 */
    SOF_STAGE_SORT,       /* sort nodes of 65..8192 samples */
    SOF_STAGE_REDUCE,     /* best projection per node */
    SOF_STAGE_COUNT
};
/* The size classes run concurrently after the plan (the big-node stages on
 * one auxiliary stream of the context, MID2 then SORT on another, MID then
 * SMALL on the caller's stream), and REDUCE after all of them.  While timing
 * is enabled, every sof_find_splits call records HIP events before and after
 * each stage on the stream that runs it, and around the whole sequence
 * (events are created on first use, so enabling is not for graph capture).
 * sof_timing_read waits for the recorded events and writes summed
 * milliseconds since the last read: ms[s] for stage s (from its start to its
 * end on its stream, so concurrent stages overlap and their sum exceeds the
 * whole) and ms[SOF_STAGE_COUNT] for the whole sequence (ms holds
 * SOF_STAGE_COUNT + 1 floats), and the number of calls.  Errors:
 * SOF_ERR_INVALID_ARG for NULL arguments, SOF_ERR_HIP if an event query
 * fails. */
/* enable: 0 off, 1 on, 2 on with the size classes run one after another on
 * the caller's stream (no fork), so that each stage's events bound its own
 * kernels alone, 3 on with only the events around the whole sequence (the
 * stage figures read 0; the least added work per call); for measurement
 * only. */
int sof_timing_enable(sof_ctx* ctx, int enable);
int sof_timing_read(sof_ctx* ctx, float* ms, int32_t* calls);

#ifdef __cplusplus
}
#endif
#endif /* SOF_H */
