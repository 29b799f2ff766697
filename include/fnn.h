/*
 * fnn.h -- C ABI of the MI355X epsilon-graph library.
 *
 * Exact fixed-radius near-neighbour graphs in a general metric space with a
 * cover tree (Raulet, Morozov, Buluc, Yelick, "Distributed-Memory Parallel
 * Algorithms for Fixed-Radius Near Neighbor Graph Construction").
 *
 * Problem statement (Definitions): a finite point set P with a metric d and a
 * threshold eps > 0; the epsilon-graph has an edge (p, q) for every pair with
 * d(p, q) <= eps.  This library returns it as a symmetric CSR over the input
 * indices.  Two calls do the work: a batched, level-by-level cover-tree
 * build (Section IV-A, Algorithms 1 and 2) and an all-points range query
 * over that tree (Section IV-B, Algorithm 3, with query batches).
 *
 * Conventions
 *  - Plain C, no C++ or framework types cross this boundary.
 *  - Pointers documented as "device" are HIP device pointers on the current
 *    device; "host" pointers are ordinary host memory.
 *  - Every call returns FNN_OK (0) or a negative error code; on error the
 *    output handle is set to NULL, nothing leaks, and fnn_last_error()
 *    returns a message (thread-local).
 *  - Work is enqueued on the calling thread's bound stream (fnn_set_stream;
 *    default: the null stream).  fnn_tree_build and fnn_eps_graph return
 *    after their results are complete on that stream (they synchronize on
 *    it, since sizes are data dependent).
 *  - Library-owned memory is released with fnn_free.
 */
#ifndef FNN_H
#define FNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Metrics (Definitions: Euclidean, cosine, Hamming and edit distance are
 * the metrics the paper names; "cosine" is taken as the angle, which is a
 * metric, and edit distance as unit-cost Levenshtein). */
typedef enum {
    FNN_L2 = 0,          /* float32 rows [n x dim]; finite, |x| <= B(dim) =   */
                         /* min(1e16, sqrt(1e37 / dim)), else EUNSUPPORTED    */
    FNN_ANGULAR = 1,     /* float32 rows [n x dim], no zero row, same bound   */
    FNN_HAMMING = 2,     /* uint64 rows [n x dim/64]; dim = bits, % 64 == 0   */
    FNN_LEVENSHTEIN = 3  /* uint8 rows [n x dim]; dim = row stride in bytes,  */
                         /* symbols 0..254, padded with 0xFF; length = index  */
                         /* of the first 0xFF (or dim); dim <= 256            */
} fnn_metric;

/* Error codes. */
enum {
    FNN_OK = 0,
    FNN_EINVAL = -1,        /* bad argument (NaN/Inf coordinate, eps <= 0,  */
                            /* dim rules, zero angular row, NULL pointer)    */
    FNN_ENOMEM = -2,        /* device or host allocation failed              */
    FNN_EHIP = -3,          /* a HIP runtime call failed                     */
    FNN_EUNSUPPORTED = -4,  /* valid input outside what the kernels support  */
    FNN_EINTERNAL = -5      /* an internal consistency check failed          */
};

/* Leaf-tile arithmetic of the query. */
typedef enum {
    FNN_PREC_FP32 = 0,   /* direct-difference FP32 tiles (the plain path)      */
    FNN_PREC_BF16 = 1,   /* MFMA BF16 Gram filter, FP32 recompute of survivors */
    FNN_PREC_FP8 = 2,    /* MFMA FP8 (E4M3) Gram filter, FP32 recompute        */
    FNN_PREC_I8 = 3,     /* Hamming codes of <= 256 bits: exact int8 MFMA Gram */
                         /* (bits as +-1 bytes: s.t = K - 2 d over K bits)     */
    FNN_PREC_AUTO = 4,   /* chosen per query: I8 for Hamming codes of <= 256  */
                         /* bits; FP16 for L2 / angular with 16 <= dim <= 128 */
                         /* when the filter's margin is small against eps^2   */
                         /* (2 c1 mean|x - mu|^2 <= eps^2 / 2, mu per cloud); */
                         /* FP32 tiles otherwise (stats: precision_used)      */
    FNN_PREC_FP16 = 5    /* MFMA FP16 Gram filter on rows scaled by a power   */
                         /* of two (largest |coordinate| in [2^14, 2^15)):   */
                         /* the BF16 filter with an 8x narrower margin        */
} fnn_precision;

/* How CSR rows are sized. */
typedef enum {
    FNN_SCHED_TWO_PASS = 0,  /* count pass, scan, fill pass (always exact)     */
    FNN_SCHED_LEARNED = 1    /* cost-model pre-sized slots, one pass; rows that */
                             /* overflow fall back to the two-pass path         */
} fnn_sched;

/* Options for the _ex calls.  Zero-initialise, set struct_size, then set the
 * fields to change; a zero field keeps its default. */
typedef struct fnn_options {
    int32_t struct_size;  /* sizeof(fnn_options)                             */
    int32_t zeta;         /* leaf size (Algorithm 2); default 64             */
    int32_t pack;         /* points per query/leaf tile block; default 64
                             (Levenshtein: 1, one leaf block per pack)       */
    int32_t precision;    /* fnn_precision; default FNN_PREC_FP32.  BF16,    */
                          /* FP16 and FP8 apply to L2 / angular with dim <=  */
                          /* 128 (else FNN_EUNSUPPORTED), I8 to Hamming codes */
                          /* of <= 256 bits (else FNN_EUNSUPPORTED); BF16 /   */
                          /* FP16 / FP8 on integer metrics run the plain tiles */
    int32_t sched;        /* fnn_sched; default FNN_SCHED_TWO_PASS           */
    int32_t validate;     /* 1: also measure the max FP32 distance error     */
                          /* against FP64 and count filter false negatives    */
    int32_t kmax;         /* candidates examined per net-selection pass     */
                          /* and hub (1..256; default 64)                   */
    int32_t trace;        /* 1: keep per-point features and targets of this  */
                          /* query for training the cost model               */
    int32_t slack_pct;    /* learned schedule: slot slack in percent of the  */
                          /* predicted row length (default 30; may be < 0)   */
    int32_t graph_passes; /* build: net-selection passes recorded into one  */
                          /* hipGraph and replayed between host checks;     */
                          /* query: traversal levels recorded the same way  */
                          /* over device-resident frontier queues (a level  */
                          /* that may not fit stops them; eager levels      */
                          /* finish).  Default 4, rounded up to even; 1 =   */
                          /* one eager pass / level per host check          */
    int32_t proj;         /* BF16 / FP8 filter on the K leading principal    */
                          /* coordinates (a conservative bound: |Q^T(x-y)|   */
                          /* <= ||Q|| |x-y|): 0 = K the smallest multiple of */
                          /* 16 with twice the residual variance <= eps^2/2, */
                          /* if below the padded dim, else none (default);   */
                          /* -1 = none; 16..128 in steps of 16 = that K;     */
                          /* else EINVAL                                     */
    int32_t list_cap;     /* initial capacity (entries) of the MFMA filter's */
                          /* survivor list, of the plain tiles' edge list   */
                          /* and of the traversal's replayed frontier and   */
                          /* interaction buffers; 0 = automatic (default).  */
                          /* A list that overflows is redone: the filter    */
                          /* runs again into a list sized from its count,   */
                          /* the tiles fall back to the count / fill pair   */
                          /* of passes, the traversal finishes eagerly.     */
                          /* Results never depend on it; small values force */
                          /* those paths (tests).                           */
    int32_t lpt;          /* learned schedule: 1 = the tile pass takes its   */
                          /* pack pairs in LPT order of predicted cost,     */
                          /* heaviest first, each work-group the next as it */
                          /* finishes (Graham's rule, which the paper uses  */
                          /* to place cells, Section IV-D); default 0: list */
                          /* order, grid stride (measured faster)           */
    int32_t reserved[3];
} fnn_options;

typedef struct fnn_tree fnn_tree;  /* opaque; device-resident cover tree */

/* Symmetric CSR result.  Rows are the input indices 0..n-1; each row lists
 * its neighbours' input indices in ascending order, no self loops, and
 * dist[k] is the FP32 distance (within 1e-5 relative of FP64).  Arrays are
 * device memory owned by the library. */
typedef struct fnn_csr {
    uint32_t kind;        /* library tag; do not modify                      */
    uint32_t pad_;
    int64_t n;
    int64_t nnz;
    int64_t *row_ptr;     /* device, n + 1                                   */
    int32_t *col;         /* device, nnz                                     */
    float *dist;          /* device, nnz                                     */
} fnn_csr;

/* Counters and timings of the last build or query on a handle. */
typedef struct fnn_stats {
    int64_t n;
    int64_t nodes;            /* cover-tree vertices                         */
    int64_t leaf_blocks;      /* leaf vertices holding <= zeta points        */
    int64_t packs;            /* query tile blocks                           */
    int64_t rounds;           /* build levels processed                      */
    int64_t netsel_passes;    /* net-selection passes over all hubs          */
    int64_t build_dist_evals; /* metric evaluations in the build             */
    int64_t traverse_tests;   /* node-pair tests in the traversal            */
    int64_t interactions;     /* block pairs sent to leaf tiles              */
    int64_t tile_pairs;       /* point pairs evaluated in leaf tiles (once   */
                              /* per unordered pair, per pass)               */
    int64_t filter_pairs;     /* pairs screened by the MFMA filter           */
    int64_t filter_survivors; /* pairs the filter passed to FP32             */
    int64_t fp64_rechecks;    /* borderline pairs decided in FP64            */
    int64_t edges;            /* nnz (ordered pairs)                          */
    int64_t overflow_rows;    /* learned schedule: rows re-done in two pass  */
    int64_t validate_mismatch;/* validate: filter false negatives (must be 0)*/
    int64_t spilled;          /* learned: entries past their predicted slots */
    double max_rel_err;       /* validate: max |dist32 - dist64| / dist64    */
    double build_ms, traverse_ms, tile_ms, count_ms, scan_ms, fill_ms,
           sort_ms, total_ms;
    double pred_mae;          /* learned: mean |predicted - true| log1p(deg) */
    double pred_sum_ratio;    /* learned: sum predicted / sum true degrees    */
    double filter_ms;         /* MFMA filter kernel alone (last launch)       */
    int64_t proj_dim;         /* principal coordinates the filter used (0:   */
                              /* the coordinates themselves)                 */
    double proj_captured;     /* their share of the variance                  */
    int64_t precision_used;   /* fnn_precision the query ran with            */
    int64_t landmark_cells;   /* landmark mode: Voronoi cells                */
    int64_t landmark_rows;    /* landmark mode: cell members + ghosts        */
    double landmark_partition_ms; /* centres, cells, ghosts, gathered rows    */
    double landmark_forest_ms;    /* per-cell forest build and self-join      */
    double landmark_merge_ms;     /* pairs kept once, rows mapped and sorted  */
    int64_t launches;         /* kernels launched eagerly by the call         */
    int64_t graph_launches;   /* recorded launch sequences replayed           */
    int64_t graph_kernels;    /* kernels those replays ran                    */
    int64_t fill_path;        /* how the CSR was filled: 0 row cursors (or    */
                              /* the learned slots), 1 the survivor ranks     */
                              /* with column and distance stores, 2 the ranks */
                              /* with packed words that the row sort unpacks  */
} fnn_stats;

/* Build the cover tree of n points (Algorithms 1-2).  points: device
 * pointer, layout per metric above, caller-owned, only read during the
 * call (the tree keeps its own permuted copy).  n >= 1.  On success *out
 * receives a library-owned tree. */
int fnn_tree_build(const void *points, int64_t n, int32_t dim,
                   fnn_metric metric, fnn_tree **out);
int fnn_tree_build_ex(const void *points, int64_t n, int32_t dim,
                      fnn_metric metric, const fnn_options *opt,
                      fnn_tree **out);

/* All-points range query: every ordered pair (i, j), i != j, with
 * d(p_i, p_j) <= eps, as a symmetric CSR (Definitions; Algorithm 3 run for
 * query batches).  eps must be finite and > 0; Hamming and Levenshtein use
 * floor(eps).  The edge set equals the FP64 reference predicate exactly. */
int fnn_eps_graph(const fnn_tree *tree, double eps, fnn_csr **out);
int fnn_eps_graph_ex(const fnn_tree *tree, double eps,
                     const fnn_options *opt, fnn_csr **out);

/* Bichromatic range query: every pair (q, p), q a row of `queries`, p a point
 * of `tree`, with d(q, p) <= eps (the query of foreign points against a local
 * tree that Algorithms 4-6 run on each rank; here on one GPU).  queries:
 * device pointer, nq rows in the tree's metric layout and dim, caller-owned,
 * only read during the call.  The queries get a cover tree of their own
 * (built with `opt`); Algorithm 3 then runs on the pair of trees, visiting
 * only pairs across them.  *out: CSR with nq rows (query order), columns =
 * the tree's input indices, ascending, dist as in fnn_eps_graph; the same
 * exactness.  The tree must hold one cloud (FNN_EUNSUPPORTED for a batch);
 * the learned schedule and traces are not available (FNN_EUNSUPPORTED);
 * eps must be finite and > 0 (FNN_EINVAL).  Stats (fnn_get_stats on the
 * CSR) count the query tree's build as well. */
int fnn_eps_query(const fnn_tree *tree, const void *queries, int64_t nq, double eps,
                  const fnn_options *opt, fnn_csr **out);

/* ---- many independent clouds in one batch ---------------------------------
 * The level-synchronous build (Algorithm 2 processes every hub of a level
 * together) and the batched query (Algorithm 3 over query batches) extend to
 * a forest: each cloud gets its own cover tree, and the hubs and vertex
 * pairs of all clouds share every kernel launch.  This is also the shape of
 * the per-cell trees of the landmark partitioning (Section IV-D).
 *
 * fnn_tree_build_batch: points holds the rows of all clouds back to back
 * (device, layout per metric, one dim for all); cloud c is rows
 * [offsets[c], offsets[c+1]).  offsets: host array of nclouds + 1 values,
 * offsets[0] = 0, non-decreasing; empty clouds are allowed, but the total
 * must be >= 1.  The handle works with every tree call; in fnn_tree_export
 * of a batch of two or more non-empty clouds, vertex 0 is a virtual root
 * (radius +inf) whose children are the cloud roots in cloud order.
 *
 * fnn_eps_graph_batch: eps is a host array of nclouds thresholds (entries of
 * empty clouds are ignored).  The result is one symmetric CSR over all rows
 * (global row indices): cloud c's rows hold exactly the eps[c]-graph of
 * cloud c; no edge joins two clouds.  fnn_eps_graph on a batch tree applies
 * one eps to every cloud. */
int fnn_tree_build_batch(const void *points, const int64_t *offsets,
                         int32_t nclouds, int32_t dim, fnn_metric metric,
                         const fnn_options *opt, fnn_tree **out);
int fnn_eps_graph_batch(const fnn_tree *tree, const double *eps,
                        int32_t nclouds, const fnn_options *opt,
                        fnn_csr **out);

/* ---- autotuner ------------------------------------------------------------
 * Times the whole path (build + query, wall clock, median of `reps` runs
 * after one untimed run) under candidate options on the caller's input and
 * returns the fastest.  Candidates differ only in options that never change
 * the graph: filter precision (FP32 / BF16 for vector metrics with
 * dim <= 128, FP32 / I8 for Hamming codes of <= 256 bits), schedule
 * (two-pass / learned, when a cost model is installed), zeta in
 * {32, 64, 128}, kmax in {32, 64, 128}, the tile block size pack in
 * {32, 64} (not for strings), the net-selection passes per graph replay
 * graph_passes in {2, 4, 8} (the granularity of the build's device queue)
 * and, for the learned schedule, lpt in {0, 1}; searched by coordinate
 * descent from `base` (NULL: defaults; its trace and validate are
 * ignored).  points / offsets / nclouds / dim / metric / eps as in
 * fnn_tree_build_batch and fnn_eps_graph_batch (one cloud: offsets =
 * {0, n}).  Answers are cached in-process per (metric, dim, log2 n,
 * log2 nclouds, base zeta / pack / kmax / graph_passes / precision / sched
 * / proj / lpt); a cached answer is returned at once with cached = 1.
 * fnn_autotune_clear empties the cache. */
typedef struct fnn_tune_result {
    fnn_options best;     /* fastest options found                           */
    double best_ms;       /* their median build + query time                 */
    double base_ms;       /* the base options' median time                   */
    int32_t ncand;        /* option sets timed                               */
    int32_t cached;       /* 1: answer from the cache, nothing was timed     */
    double reserved[4];
} fnn_tune_result;

int fnn_autotune(const void *points, const int64_t *offsets, int32_t nclouds,
                 int32_t dim, fnn_metric metric, const double *eps,
                 const fnn_options *base, int32_t reps, fnn_tune_result *out);
void fnn_autotune_clear(void);

/* ---- landmark mode (Section IV-D, Algorithm 5; Section IV-E, Lemma 1 and
 * Algorithm 6), on one GPU ----------------------------------------------------
 * The same epsilon-graph as fnn_tree_build + fnn_eps_graph, assembled the
 * way the paper's landmark algorithm does: `ncells` centres drawn from the
 * points (seeded), the Voronoi cells of those centres, each cell's
 * eps-ghosts (points of other cells p with d(p, c_i) <= d(p, C) + 2 eps,
 * Lemma 1; widened by the FP32 rounding bound, so no ghost is missed), one
 * cover tree per cell over its members and ghosts (built and queried as one
 * batch), and every ordered pair kept once.  points / n / dim / metric as in
 * fnn_tree_build (device, caller-owned, read during the call); eps as in
 * fnn_eps_graph; ncells >= 1 (capped at n); opt applies to the per-cell
 * build and query (traces are not available: FNN_EUNSUPPORTED).  *out: the
 * symmetric CSR over the input indices, identical to fnn_eps_graph's.
 * Stats: landmark_cells, landmark_rows (members + ghosts), phase times.
 * FNN_EUNSUPPORTED when members + ghosts exceed 2^30 - 1 rows, or when a
 * row is not a multiple of 4 bytes (strings: dim % 4 != 0). */
int fnn_landmark_eps_graph(const void *points, int64_t n, int32_t dim,
                           fnn_metric metric, double eps, int32_t ncells,
                           uint64_t seed, const fnn_options *opt, fnn_csr **out);

/* Release a fnn_tree* or fnn_csr* (NULL is ignored). */
void fnn_free(void *handle);

/* Stream for this thread's later calls (a hipStream_t; NULL = null stream). */
int fnn_set_stream(void *stream);

/* Optional device allocator (problem statement: the caller owns the memory
 * system).  Once set, every device buffer of a call comes from it: the arrays
 * handed back (tree and CSR arrays, released by fnn_free) and the call's
 * scratch chunks (taken in pieces of at least 256 MB and returned before the
 * call returns, after the stream has drained).  alloc returns a device
 * pointer (256-byte aligned) or NULL; NULL makes the call fail with
 * FNN_ENOMEM and free everything it took.  Not routed through it: the
 * installed cost model's 21 KB device copy and the fixed array of
 * fnn_mlp_loss_grad_noalloc.  Passing NULL functions restores hipMalloc /
 * hipFree and the library's own cache of scratch chunks. */
typedef void *(*fnn_alloc_fn)(size_t bytes, void *ctx);
typedef void (*fnn_free_fn)(void *ptr, void *ctx);
int fnn_set_allocator(fnn_alloc_fn alloc, fnn_free_fn free_, void *ctx);

/* Copy the counters of the last operation on a tree or CSR handle. */
int fnn_get_stats(const void *handle, fnn_stats *out);

/* Debug export of the cover tree to caller-provided host arrays.
 * fnn_tree_info gives the sizes; fnn_tree_export fills:
 *   order[n]        input index of each point in tree order
 *   center[nodes]   input index of each vertex's point
 *   radius[nodes]   stored radius (an upper bound on d(center, x) over the
 *                   vertex's points)
 *   level[nodes]    split level (children lie within 2^level of the centre,
 *                   sibling centres are more than 2^(level-1) apart)
 *   child_begin/child_count[nodes]  children are consecutive vertex ids
 *   pt_begin/pt_end[nodes]          the vertex's points are
 *                                   order[pt_begin .. pt_end)
 * A vertex with child_count == 0 is a leaf block: its points are leaves. */
int fnn_tree_info(const fnn_tree *tree, int64_t *n, int64_t *nodes);
int fnn_tree_export(const fnn_tree *tree, int32_t *order, int32_t *center,
                    float *radius, int32_t *level, int32_t *child_begin,
                    int32_t *child_count, int32_t *pt_begin, int32_t *pt_end);

/* ---- learned cost model (schedules only; never decides an edge) ----------
 * A 16 -> 64 -> 64 -> 2 perceptron with SiLU activations predicts, per point,
 * log1p(block pairs of its query pack) and log1p(its neighbour count) from
 * scale-free tree features.  Parameters: 5378 floats, row-major
 * W1[64][16], b1[64], W2[64][64], b2[64], W3[2][64], b3[2].  Loss of a batch
 * of B samples: (1/(2B)) * sum of squared errors over both outputs. */
#define FNN_MLP_NPARAMS 5378
#define FNN_MLP_NFEAT 16

/* Install the model used by FNN_SCHED_LEARNED (host array of
 * FNN_MLP_NPARAMS floats, copied). */
int fnn_set_cost_model(const float *params, int64_t nparams);

/* Trace of a query run with options.trace = 1: device arrays, owned by the
 * CSR handle, in tree order: features [n][16], targets [n][2]. */
int fnn_get_trace(const fnn_csr *csr, const float **features,
                  const float **targets, int64_t *n);

/* Inference: Y[n][2] = f(X[n][16]); all device pointers. */
int fnn_mlp_forward(const float *params, const float *X, int64_t n, float *Y);

/* Full-batch loss and its gradient (device params/X/T/grad; *loss on host). */
int fnn_mlp_loss_grad(const float *params, const float *X, const float *T,
                      int64_t n, float *grad, double *loss);

/* Allocation-free variant of fnn_mlp_loss_grad, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same loss and gradient; params, X, T,
 * grad and *loss are all DEVICE pointers (loss: one double, the mean loss),
 * caller-owned.  Nothing is allocated and nothing waits on the stream: the
 * work is enqueued on the bound stream and the results are valid once it
 * completes.  Partial sums live in a fixed per-device array of the library
 * (5.5 MB, held until the process ends): at most 256 work-groups, each
 * owning one row of partial gradients and one partial loss, then reduced in
 * a fixed order, so repeated calls on the same input give identical bits.
 * Every call on a device shares that array, so calls that overlap on one
 * device (two streams, two threads) race: serialize them.  n must be at
 * most FNN_NOALLOC_MAX_SAMPLES, else FNN_EINVAL. */
#define FNN_NOALLOC_MAX_SAMPLES (((int64_t)1) << 31)
int fnn_mlp_loss_grad_noalloc(const float *params, const float *X, const float *T,
                              int64_t n, float *grad, double *loss);

/* Train in place with Adam (device params, X, T): `epochs` passes over a
 * seeded shuffle in batches of `batch`; epoch_loss (host, may be NULL)
 * receives the mean loss of each epoch. */
int fnn_mlp_train(float *params, const float *X, const float *T, int64_t n,
                  int32_t epochs, int32_t batch, float lr, uint64_t seed,
                  double *epoch_loss);

/* Message of the last error on this thread ("" if none). */
const char *fnn_last_error(void);

/* ABI version (major * 10000 + minor * 100 + patch). */
int fnn_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FNN_H */
