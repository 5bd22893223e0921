/*
 * nnm.h -- C ABI of the MI355X (gfx950) nearest-neighbour clustering library.
 *
 * The library computes the clustering of N records with D features by the
 * nearest neighbour method (single linkage) exactly, on one GPU:
 *
 *   knn_build    the exact k nearest neighbours of every point;
 *   mst_build    the minimum spanning tree of the complete graph on the
 *                points (the single-linkage merge tree), sorted by key;
 *   cluster_cut  the constrained cut of that tree into clusters.
 *
 * Definitions (shared by every entry point):
 *
 *   Pair distance: eq. (1) of the paper, rho = sqrt(sum_j (x_j1 - x_j2)^2).
 *   The library orders pairs by the squared distance s, evaluated in IEEE
 *   FP64 as follows: every FP32 feature is widened exactly to FP64, the
 *   per-feature difference and its square are each rounded once and the
 *   squares are added left to right over features 0..D-1 (no fused
 *   multiply-add).  The reported distance is w = sqrt(s), correctly rounded.
 *
 *   Key: pairs are compared by (s, min(i,j), max(i,j)), lexicographically.
 *   All keys are distinct, so the minimum spanning tree is unique.
 *
 *   Merge tree: the section "General description of the algorithm for
 *   constructing the set of minimum distances" unites clusters along the
 *   globally smallest pairs, skipping pairs already inside one cluster,
 *   until clustering ends.  Run to the end that process yields the
 *   key-ordered minimum spanning tree; mst_build returns its N-1 edges.
 *
 *   Constraints: section "Problem settings" (KL1..KL4) and the distance
 *   threshold of the "Problem statement"; see cluster_cut below.
 *
 * Conventions:
 *   - Every pointer named *_dev is device memory on the current HIP device;
 *     *_host is host memory.  The caller allocates and owns every buffer,
 *     including the workspace; the library allocates nothing.
 *   - `stream` is a hipStream_t (NULL = the default stream).  GPU entry
 *     points enqueue their work on it and return once the results are
 *     complete on the device (they synchronise on `stream` internally,
 *     because the number of rounds is data-dependent).
 *   - X_dev is FP32 row-major: feature f of point i at X_dev[i * ld + f].
 *   - Failures return a negative nnm_status and leave outputs undefined;
 *     argument checks happen before any device work.
 */
#ifndef NNM_H
#define NNM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NNM_OK = 0,
    NNM_EINVAL = -1,        /* bad size, null pointer, short workspace        */
    NNM_ENOMEM = -2,        /* (not raised: the library allocates nothing)    */
    NNM_EDEVICE = -3,       /* a HIP call failed                              */
    NNM_ENONFINITE = -4,    /* a feature is NaN or infinite                   */
    NNM_EUNSUPPORTED = -5,  /* precision not usable for these inputs          */
    NNM_ETOOLARGE = -6      /* input needs more than the fixed scratch of
                               mst_build_noalloc                              */
} nnm_status;

/*
 * Precision of the candidate pass.  Every precision gives the same, exact
 * result: candidates within a proven error bound of the selection threshold
 * are rescored in FP64 by the definition above.
 *   FP32  direct differences on the vector ALUs (D <= 32);
 *   BF16  x.y form on the matrix cores, FP32 accumulation (D <= 26);
 *   FP16  as BF16 with FP16 operands (D <= 26);
 *   FP8   e4m3 operands; only for integer features in [-16, 16] (D <= 26);
 *   AUTO  FP8 for such integer data, else FP16 when D <= 26, else FP32.
 * BF16 / FP16 / FP8 also return NNM_EUNSUPPORTED for data whose feature
 * ranges would need a scale factor outside 2^-60 .. 2^60 (AUTO then uses
 * FP32).
 */
typedef enum {
    NNM_PREC_FP32 = 0,
    NNM_PREC_BF16 = 1,
    NNM_PREC_FP8 = 2,
    NNM_PREC_AUTO = 3,
    NNM_PREC_FP16 = 4
} nnm_precision;

/* One tree edge: u < v, s = FP64 squared distance, w = sqrt(s). 24 bytes. */
typedef struct {
    int32_t u;
    int32_t v;
    double s;
    double w;
} nnm_edge;

/*
 * Settings of the constrained cut ("Problem settings"; threshold from the
 * "Problem statement").  Edges are taken one at a time:
 *   kl1_max_clusters  stop once #clusters <= kl1 (<= 0: off);
 *   kl2_max_size      do not unite when the larger side has more than kl2
 *                     points (< 0: off); united clusters may exceed kl2;
 *   kl3_max_merged    do not unite when both sides hold more than kl3
 *                     points together (< 0: off);
 *   kl4_min_size      (> 1: on) first unite along edges whose smaller side
 *                     has fewer than kl4 points, in key order, re-checked
 *                     each time an edge is taken;
 *   dmax              do not unite along an edge with w > dmax (+inf: off).
 */
typedef struct {
    int64_t kl1_max_clusters;
    int64_t kl2_max_size;
    int64_t kl3_max_merged;
    int64_t kl4_min_size;
    double dmax;
} nnm_cut_params;

/* Run options.  Zero-initialised options mean "defaults". */
typedef struct {
    int32_t precision;      /* nnm_precision (0 = FP32; use AUTO for auto)   */
    int32_t knn_k;          /* cache depth, 1..32 (0: 6; FP32: 8)             */
    int32_t survivor_cap;   /* candidates kept per row, 16..2048 (0 = auto)   */
    int32_t disable_prune;  /* 1: rescan every exhausted row (debug)          */
    int32_t force_fallback; /* 1: rescore every row by a full FP64 scan       */
    int32_t col_splits;     /* column splits per row tile (0 = auto)          */
    int32_t fixed_chunks;   /* 1: column chunks never follow the components
                               (debug)                                        */
    int32_t graph;          /* 1: the merge rounds after the first run as one
                               captured hipGraph, replayed once per round
                               (launch sizes taken on the device, one host
                               read per round); the graph is kept for later
                               calls with the same buffers, sizes and
                               settings.  Results are identical.             */
    int32_t split_target0;  /* workgroups the column splits aim at in the
                               first round (0: 4096)                          */
    int32_t split_target;   /* ... and in the bounded scans of later rounds
                               (0: 8192)                                      */
    int32_t metric;         /* nnm_metric (0: Euclidean, eq. (1))            */
    int32_t reserved[5];
} nnm_options;

/*
 * The pair metric ("Overall idea of the algorithm": another metric may take
 * the place of eq. (1)).  Keys and reported distances w:
 *   EUCLIDEAN  s = the squared distance above, w = sqrt(s);
 *   L1         s = sum over f of |x_f - y_f| (each term exact in FP64, added
 *              left to right), w = s;
 *   LINF       s = max over f of |x_f - y_f| (exact), w = s;
 *   COSINE     every row is first scaled to unit Euclidean length (norm: the
 *              square root of the FP64 sum of squares in feature order;
 *              each feature divided by it in FP64 and rounded once to FP32;
 *              a zero row stays zero), then EUCLIDEAN on those rows:
 *              w = sqrt(2 - 2 cos) up to that rounding.
 * L1 and LINF have no dot-product form: their candidates always come from
 * the FP32 vector path (AUTO picks it; BF16 / FP16 / FP8 give
 * NNM_EUNSUPPORTED).  Pairs are ordered by (s, min index, max index) in
 * every metric.
 */
typedef enum {
    NNM_METRIC_EUCLIDEAN = 0,
    NNM_METRIC_L1 = 1,
    NNM_METRIC_LINF = 2,
    NNM_METRIC_COSINE = 3
} nnm_metric;

/* Per-call measurements (all optional to read; filled when non-NULL). */
typedef struct {
    int32_t precision_used;     /* nnm_precision actually used                */
    int32_t integer_mode;       /* 1: candidate distances were exact          */
    int32_t rounds;             /* merge rounds (mst_build)                   */
    int32_t knn_k;              /* cache depth used                           */
    int64_t rows_scanned;       /* rows sent through the candidate pass       */
    int64_t pairs_evaluated;    /* candidate pairs evaluated (tiles run)      */
    int64_t survivors;          /* candidates rescored in FP64                */
    int64_t overflow_rows;      /* rows that needed the exact full FP64 scan  */
    double max_abs_err;         /* max |t - s| over rescored candidates       */
    double max_rel_err;         /* max |t - s| / s over candidates with s > 0 */
    double max_bound;           /* largest bound E(t) on |t - s| that the
                                   candidate pass applied to a rescored
                                   candidate (0 on exact integer data)        */
    double ms_total;            /* wall time of the call, ms                  */
    double ms_candidates;       /* candidate kernels, ms (HIP events)         */
    double ms_rescore;          /* FP64 rescoring, ms                         */
    double ms_merge;            /* cursor, component minima, union-find, ms   */
    double ms_sort;             /* edge and component sorts, ms               */
    int64_t rows_per_round[32]; /* rows scanned in each round                 */
    int64_t comps_per_round[32];/* components at the start of each round      */
    int64_t cand_launches;      /* candidate-kernel launches                  */
    int64_t rescanned_bounded;  /* overflowed rows scanned again below a bound */
    int64_t pairs_per_round[32];/* candidate pairs evaluated in each round    */
    int64_t over_per_round[32]; /* survivor-list overflows in each round      */
    int64_t exact_per_round[32];/* rows needing the exact scan in each round  */
    double cand_ms_per_round[32];/* candidate-kernel time in each round, ms    */
    int64_t surv_per_round[32]; /* survivors rescored in each round           */
    double max_err_ratio;       /* max over rescored candidates of |t - s| /
                                   E(t), E(t) the bound applied to it (0/0 = 0,
                                   x/0 = inf); the proof makes it <= 1        */
    double ms_graph;            /* graph-replayed rounds (options.graph), ms;
                                   their kernels are not in the phase times
                                   above, nor in the per-round overflow and
                                   candidate-time entries                     */
    int32_t graph_rounds;       /* rounds run by replaying the graph          */
    int32_t graph_nodes;        /* kernel nodes of the round graph            */
    int32_t graph_captured;     /* 1: this call captured the graph (0: it was
                                   kept from an earlier call)                 */
    int32_t pad_;
} nnm_report;

/* Fill *opt with the defaults (AUTO precision, automatic k and caps). */
void nnm_default_options(nnm_options *opt);

/* Human-readable text of a status code (static storage). */
const char *nnm_strerror(int32_t status);

/*
 * Workspace bytes that mst_build needs for n points of d features with
 * these options (NULL = defaults).  Returns NNM_EINVAL for n < 1,
 * d < 1 or d > 32.
 */
nnm_status mst_workspace_size(int64_t n, int32_t d, const nnm_options *opt,
                              size_t *bytes);

/* Workspace bytes that knn_build needs for n points, d features, depth k. */
nnm_status knn_workspace_size(int64_t n, int32_t d, int32_t k,
                              const nnm_options *opt, size_t *bytes);

/*
 * Exact k nearest neighbours of every point by key (s, j), j != i
 * (the selection of minimum distances of the section "Overall idea of the
 * algorithm", one row at a time).
 *   X_dev     [n][ld] FP32, device, read only;
 *   k         1..32;
 *   idx_dev   [n][k] int32, device: neighbour indices, ascending key;
 *   s_dev     [n][k] FP64, device: their squared distances;
 *   len_dev   [n] int32, device: min(k, n-1) valid entries per row;
 *             entries past len are idx = -1, s = +inf.
 * Errors: NNM_EINVAL (n < 1, d < 1, d > 32, ld < d, k out of range, null
 * pointer, ws_bytes short), NNM_ENONFINITE (a NaN/Inf feature),
 * NNM_EUNSUPPORTED (precision unusable for these inputs).
 */
nnm_status knn_build(const float *X_dev, int64_t n, int32_t d, int64_t ld,
                     int32_t k, const nnm_options *opt, void *ws_dev,
                     size_t ws_bytes, int32_t *idx_dev, double *s_dev,
                     int32_t *len_dev, void *stream, nnm_report *rep);

/*
 * The key-ordered minimum spanning tree (single-linkage merge tree).
 *   X_dev      [n][ld] FP32, device, read only;
 *   edges_dev  [n-1] nnm_edge, device: sorted ascending by key (s, u, v).
 * n = 1 gives no edges.  Errors as for knn_build.
 */
nnm_status mst_build(const float *X_dev, int64_t n, int32_t d, int64_t ld,
                     const nnm_options *opt, void *ws_dev, size_t ws_bytes,
                     nnm_edge *edges_dev, void *stream, nnm_report *rep);

/*
 * mst_build for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same tree as mst_build, with no workspace argument.  Its scratch
 * memory is a fixed device array of NNM_NOALLOC_SCRATCH_BYTES inside the
 * library (one per GPU, held from the library's first use on that GPU until
 * the process ends); the call allocates nothing and creates no HIP events,
 * so the report's phase times (ms_candidates .. ms_sort) stay 0.
 *   X_dev, n, d, ld, opt, edges_dev, stream, rep: as for mst_build.
 * Limit: inputs whose mst_workspace_size() exceeds NNM_NOALLOC_SCRATCH_BYTES
 * return NNM_ETOOLARGE before any device work (with default options up to
 * about 65,536 points of at most 26 features).
 * Every call on one GPU shares that GPU's scratch: calls that overlap on one
 * GPU (other host threads, other streams) race and must be serialised by
 * the caller.  Errors otherwise as for mst_build.
 */
#define NNM_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
nnm_status mst_build_noalloc(const float *X_dev, int64_t n, int32_t d,
                             int64_t ld, const nnm_options *opt,
                             nnm_edge *edges_dev, void *stream,
                             nnm_report *rep);

/*
 * The same tree by the paper's own pipeline (section "General description
 * of the algorithm for constructing the set of minimum distances"): each
 * pass selects the P smallest pairs of points not inside one cluster,
 * sorts them by key and unites clusters along them in that order (pairs
 * that are inside a cluster by then are skipped), until one cluster is
 * left.  A pass costs a scan of every row; mst_build reaches the same tree
 * with far less work, and this entry point exists to measure the paper's
 * scheme on the same kernels.
 *   P          pairs per pass (0: n / 2);
 *   ws_dev     at least pminimal_workspace_size() bytes;
 *   rep        as for mst_build; rounds = passes, comps_per_round = clusters
 *              at the start of each pass, rows_per_round = pairs taken in
 *              the pass, surv_per_round = unions it made.
 * Other arguments and errors as for mst_build.
 */
nnm_status pminimal_workspace_size(int64_t n, int32_t d, const nnm_options *opt,
                                   size_t *bytes);
nnm_status mst_build_pminimal(const float *X_dev, int64_t n, int32_t d,
                              int64_t ld, int64_t P, const nnm_options *opt,
                              void *ws_dev, size_t ws_bytes,
                              nnm_edge *edges_dev, void *stream,
                              nnm_report *rep);

/* One instance of a batched call. */
typedef struct {
    const float *X_dev;     /* [n][ld] FP32 device                             */
    int64_t n;
    int32_t d;
    int32_t pad_;
    int64_t ld;
    nnm_edge *edges_dev;    /* [n-1] device output, sorted by key              */
} nnm_instance;

/*
 * Many independent instances of uneven n and d in one call; each instance's
 * tree is exactly what mst_build gives for it alone.  The instances are
 * processed together: one launch per phase of the merge rounds serves all of
 * them (the paper's aim of keeping the GPU loaded with many uneven tasks,
 * section "Overall idea of the algorithm").
 *   inst   [count] host array of instance descriptors (n >= 1, 1 <= d <= 32,
 *          ld >= d, X_dev non-null, edges_dev non-null when n > 1);
 *   reps   NULL, or [count] host reports: every entry receives the report of
 *          the whole call.
 * The workspace must hold mst_batched_workspace_size() bytes.
 */
nnm_status mst_batched_workspace_size(const nnm_instance *inst, int32_t count,
                                      const nnm_options *opt, size_t *bytes);
nnm_status mst_build_batched(const nnm_instance *inst, int32_t count,
                             const nnm_options *opt, void *ws_dev,
                             size_t ws_bytes, void *stream, nnm_report *reps);

/*
 * Autotuner of the run options, on the caller's own data: the paper's aim of
 * keeping the GPU fully loaded whatever the size of the task (section
 * "Overall idea of the algorithm") depends on how the work is cut, so the
 * cut is measured rather than fixed.  One instance (count = 1: mst_build on
 * inst[0]) or a batch (count > 1: mst_build_batched) is built with *base and
 * then, by coordinate descent, with each value of each knob in turn, keeping
 * a value when it is faster:
 *   knn_k          4, 6, 8, 12
 *   split_target0  2048, 4096, 8192
 *   split_target   4096, 8192, 16384
 *   graph          0, 1
 * Every trial's trees are compared with the first trial's, byte for byte.
 *   inst, count   as for mst_build_batched (edges_dev receive the trees);
 *   base          starting options (NULL = defaults; precision and the debug
 *                 knobs are kept as given);
 *   ws_dev        at least mst_autotune_workspace_size() bytes;
 *   reps          timed calls per trial (the minimum counts), 1..16, after
 *                 one untimed call;
 *   best          host output: the fastest options found;
 *   trial_ms      NULL, or host [NNM_TUNE_MAX_TRIALS]: wall time of each
 *                 trial (trial 0: *base), ms;
 *   n_trials      NULL, or host output: trials run.
 * Errors: as for mst_build / mst_build_batched; NNM_EDEVICE also when two
 * trials' trees differ.
 */
#define NNM_TUNE_MAX_TRIALS 32
nnm_status mst_autotune_workspace_size(const nnm_instance *inst, int32_t count,
                                       const nnm_options *base, size_t *bytes);
nnm_status mst_autotune(const nnm_instance *inst, int32_t count,
                        const nnm_options *base, void *ws_dev, size_t ws_bytes,
                        void *stream, int32_t reps, nnm_options *best,
                        double *trial_ms, int32_t *n_trials);

/*
 * Constrained cut of a sorted tree (host code, synchronous).
 *   edges_host  [n-1] nnm_edge, host, sorted by key as mst_build returns;
 *   labels_host [n] int32, host output: cluster of each point, numbered
 *               0..K-1 in order of first appearance over i = 0..n-1;
 *   n_clusters  host output: K.
 * Errors: NNM_EINVAL (n < 1, null pointer, an edge with u >= v or out of
 * range, edges not sorted by key, a negative or NaN s or w, w decreasing
 * along the key order, or an edge taken by the cut whose two ends the edges
 * taken before it already connect, i.e. the edges are not a tree).
 */
nnm_status cluster_cut(const nnm_edge *edges_host, int64_t n,
                       const nnm_cut_params *params, int32_t *labels_host,
                       int64_t *n_clusters);

/*
 * The same cut on the device, for settings without size caps or priority
 * (KL2 < 0, KL3 < 0, KL4 <= 1).  Only KL1 ("Problem settings") and the
 * distance threshold ("Problem statement") can then stop a union, and since
 * w never decreases along the key order the admissible tree edges (those
 * with w <= dmax, i.e. not w > dmax) form a prefix: the clusters are the
 * components of the forest of the first m = min(prefix, n - KL1) edges
 * (KL1 <= 0: the whole prefix), found by a concurrent union-find on the GPU;
 * labels and K are those cluster_cut returns for the same edges.  The
 * tree's edges stay in device memory (as mst_build leaves them).
 *   edges_dev   [n-1] nnm_edge, device, sorted by key;
 *   ws_dev      at least cluster_cut_device_workspace_size(n) bytes
 *               (about 12 n bytes);
 *   labels_dev  [n] int32, device output: as cluster_cut's labels_host;
 *   n_clusters  host output: K;
 *   stream      as for mst_build; returns once the labels are complete.
 * Errors: NNM_EUNSUPPORTED when KL2, KL3 or KL4 is on (cluster_cut applies
 * those); NNM_EINVAL as for cluster_cut (n < 1 or above INT32_MAX, a null
 * pointer, a short workspace, malformed or unsorted edges, or a cycle among
 * the edges the cut takes); NNM_EDEVICE when a HIP call fails.
 */
nnm_status cluster_cut_device_workspace_size(int64_t n, size_t *bytes);
nnm_status cluster_cut_device(const nnm_edge *edges_dev, int64_t n,
                              const nnm_cut_params *params, void *ws_dev,
                              size_t ws_bytes, int32_t *labels_dev,
                              int64_t *n_clusters, void *stream);

/*
 * The clustering process itself under the settings, over all pairs of
 * points: the section "General description of the algorithm for
 * constructing the set of minimum distances" unites, step by step, the two
 * clusters of the smallest admissible pair of points in different clusters
 * ("Problem settings": KL1..KL4; "Problem statement": the distance
 * threshold).  A pair of clusters A, B is admissible when sqrt(s) <= dmax,
 * max(|A|, |B|) <= KL2 (KL2 < 0: off) and |A| + |B| <= KL3 (KL3 < 0: off);
 * with KL4 > 1 pairs with min(|A|, |B|) < KL4 come first (class 0), each
 * class in key order; the process stops at KL1 clusters (KL1 <= 0: off) or
 * when no pair is admissible.  With KL2 and KL3 off this is exactly
 * cluster_cut of the tree; with them on a blocked pair can be bypassed by a
 * longer pair that is not a tree edge, which only this entry point follows.
 * A cluster whose smallest outgoing tree edge is admissible takes that edge
 * (the smallest pair leaving it); only clusters whose smallest outgoing
 * tree edge is blocked search their points' neighbours.
 *   X_dev      [n][ld] FP32 device (as for mst_build);
 *   edges_host [n-1] host: the tree mst_build returned for this X_dev
 *              (another set of edges gives undefined labels);
 *   params     the settings (as for cluster_cut);
 *   k          neighbour prefix kept per point, 1..32 (0: 16), built when
 *              first needed; points that use theirs up get the next one
 *              from an exact FP64 scan over the columns admissible for their
 *              cluster;
 *   opt        candidate precision of the first prefixes (as for knn_build);
 *   ws_dev     at least allpairs_cut_workspace_size() bytes;
 *   labels_host, n_clusters: as for cluster_cut;
 *   stats      NULL, or host [5]: unions, GPU scans for next prefixes, points
 *              rescanned, k used, microseconds spent in those scans.
 * Synchronous; host memory O(n k).  Errors: as for knn_build and
 * cluster_cut (a NaN or negative dmax is NNM_EINVAL).
 */
nnm_status allpairs_cut_workspace_size(int64_t n, int32_t d, int32_t k,
                                       const nnm_options *opt, size_t *bytes);
nnm_status cluster_cut_allpairs(const float *X_dev, int64_t n, int32_t d,
                                int64_t ld, const nnm_edge *edges_host,
                                const nnm_cut_params *params,
                                int32_t k, const nnm_options *opt,
                                void *ws_dev, size_t ws_bytes, void *stream,
                                int32_t *labels_host, int64_t *n_clusters,
                                int64_t *stats);

#ifdef __cplusplus
}
#endif

#endif /* NNM_H */
