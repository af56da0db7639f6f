/*
 * pc.h - C ABI of the MI355X (gfx950) PC-stable skeleton library (libpc.so).
 *
 * The library computes the skeleton step of the order-independent PC algorithm (PC-stable) for
 * multivariate-normal data, as described in Zarebavani et al., "cuPC: CUDA-based Parallel PC
 * Algorithm for Causal Structure Learning on GPU" (IEEE TPDS 2019): the level loop of Algorithm 1
 * (Sec. 2.4), with the Gaussian CI test of Sec. 4.3 (Eq. 3-6) evaluated from the correlation matrix.
 *
 * Conventions for every entry point:
 *   - Pointers named "device" must point to GPU memory of the device the context was created on.
 *     The caller owns all buffers, including the workspace; the library never frees them.
 *   - Calls are ordered on the context's HIP stream. pc_corr is asynchronous. pc_level and
 *     pc_skeleton synchronise the stream before returning (their stop rule and statistics are
 *     read back on the host, as in Algorithm 2).
 *   - Every call returns a pc_status; nothing throws across the ABI. Inputs are never modified
 *     except the ones documented as in/out.
 *   - A context is not thread safe; use one context per host thread and stream.
 *   - Adjacency is a bit matrix: n rows of W = ceil(n/64) uint64 words, row-major; bit (j % 64) of
 *     word (i*W + j/64) is 1 iff edge (V_i, V_j) is present. It is symmetric, the diagonal and the
 *     bits past column n-1 are 0.
 *   - Data X is m x n FP64, row-major (sample r, variable a at X[r*n + a]).
 */
#ifndef PC_H
#define PC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Largest conditioning-set size a level can use. A run that would need a larger level stops
 * after level PC_MAX_LEVEL and returns PC_WARN_LEVEL_CAP. Levels up to 13 keep each conditioning
 * set's factor in registers; deeper levels factor each set cooperatively across a wavefront. */
#define PC_MAX_LEVEL 30

typedef enum {
    PC_OK = 0,
    PC_WARN_SAMPLE_LIMIT = 1,   /* stopped before level l because m - l - 3 <= 0 (Eq. 6 undefined) */
    PC_WARN_LEVEL_CAP = 2,      /* stopped after PC_MAX_LEVEL with nodes still having enough neighbours */
    PC_ERR_INVALID_ARG = -1,    /* null pointer, alpha outside (0,1), unknown option value */
    PC_ERR_SHAPE = -2,          /* n < 2 or m < 4 or n, m too large */
    PC_ERR_CONSTANT_COLUMN = -3,/* a variable has zero sample variance (correlation undefined) */
    PC_ERR_NONFINITE = -4,      /* X holds NaN or Inf */
    PC_ERR_WORKSPACE = -5,      /* ws_bytes < pc_workspace_bytes(...) */
    PC_ERR_HIP = -6,            /* a HIP runtime call failed */
    PC_ERR_UNSUPPORTED = -7,    /* work counts beyond 2^62, or a device without gfx950 */
    PC_ERR_SEPSET_CAPACITY = -8 /* more level >= 1 removals than sep->cap: the adjacency is complete
                                   and correct, the records past cap were dropped (*count holds
                                   the number that was needed) */
} pc_status;

typedef enum {
    PC_PREC_FP64 = 0,   /* C and every CI test in FP64 */
    PC_PREC_FP32 = 1,   /* C by FP32 MFMA GEMM, CI tests in FP32, borderline tests re-done in FP64 */
    PC_PREC_BF16X3 = 2  /* C by three BF16 MFMA products (hi*hi + hi*lo + lo*hi, FP32 accumulate),
                           CI tests in FP32, borderline tests re-done in FP64 */
} pc_precision;

typedef struct {
    int32_t precision;         /* pc_precision; default PC_PREC_FP32 */
    int32_t max_level;         /* last level to run; -1 = until the stop rule of Algorithm 1 */
    float margin_scale;        /* safety factor on the FP32 error band (default 2; must be >= 1) */
    int32_t force_recheck_all; /* 1: every FP32 test is re-evaluated in FP64 (precision audit) */
    int32_t lds_budget;        /* bytes of LDS a level work-group may use to stage C[N_i,N_i]
                                  (default 16384, so that several work-groups share a CU; capped
                                  near 50 KiB; 0 forces the global-memory gather path) */
    int32_t ranks_per_lane;    /* conditioning sets per lane in one work item (0 = automatic:
                                  1 at level 1, 4 at levels 2-3, 2 at 4-7, 1 above) */
    int32_t grid;              /* work-groups of the persistent level kernel (0 = automatic: as
                                  many as fit on the device at once) */
    int32_t timing;            /* bit mask of phases timed with HIP events into pc_run_stats:
                                  1 = correlation kernel (incl. level 0), 2 = level kernels,
                                  4 = compaction, 8 = FP64 re-check, 16 = standardization,
                                  32 = the level kernels of level 1 only. No phase is timed
                                  inside a captured graph. */
    int64_t recheck_cap;       /* capacity of the FP64 re-check queue in tests per level
                                  (0 = automatic: the sum of n^2/4 over the batch, at least
                                  2^17, at most 2^25), held in 16 equal slices that work-groups
                                  fill by their index, spilling to the next slice. A level whose
                                  borderline tests fill every slice stops the level loop; the
                                  library then completes that level and the levels after it in
                                  FP64 (C recomputed in FP64 from the standardized data of the
                                  workspace), so the result stays exact (pc_run_stats.fp64_from).
                                  Only the tail kernel (tail_tests), whose share of the queue is
                                  recheck_cap / problems, still returns PC_ERR_WORKSPACE. */
    int32_t graph_levels;      /* levels recorded in a captured graph (pc_batch_capture; 0 = 10).
                                  A replay whose datasets need more levels continues them on the
                                  stream in pc_graph_results. */
    int32_t tests_per_lane;    /* levels up to 13: rows with long neighbour lists get work items of
                                  fewer conditioning sets, so one lane runs about this many CI
                                  tests per item (0 = automatic: 32 when the call has no more
                                  variables in all than level-1 work-groups fit on the device,
                                  else 128) */
    int32_t tail_tests;        /* > 0: once a level of a problem (level >= 2, <= 8) has at most this
                                  many CI tests (bounded by sum C(d_i, l)(d_i - l)), that level and
                                  the following ones run in one work-group per problem instead of
                                  four launches per level; in a captured graph the tail kernel runs
                                  after the graph_levels recorded levels. 0 (default) = never. Not
                                  used with force_recheck_all or a per-edge ordering model. */
} pc_options;

/* One SepSet record, written for every edge removed at a level >= 1 (Algorithm 1: "store S").
 * i < j; S[0..level) holds the variable ids of the separating set in ascending order; the remaining
 * entries are -1. Edges removed at level 0 have the empty SepSet and get no record. */
typedef struct {
    int32_t i, j, level;
    int32_t S[PC_MAX_LEVEL];
} pc_sep_rec;

/* Device-side SepSet table. recs: device array of cap records. count: device int64 counter that
 * the library increments once per removal at a level >= 1 (zeroed by pc_skeleton; pc_level
 * appends to it). */
typedef struct {
    pc_sep_rec *recs;
    int64_t cap;
    int64_t *count;
} pc_sepset;

/* Per-run statistics (host memory). Index = level. */
typedef struct {
    int64_t tests[PC_MAX_LEVEL + 1];     /* CI tests evaluated on the GPU (level 0: n(n-1)/2) */
    int64_t removed[PC_MAX_LEVEL + 1];   /* edges removed in the level */
    int64_t rechecks[PC_MAX_LEVEL + 1];  /* tests re-evaluated in FP64 */
    int64_t items[PC_MAX_LEVEL + 1];     /* work items planned for the level */
    int64_t audit_violations[PC_MAX_LEVEL + 1]; /* force_recheck_all: FP32 decisions made outside
                                                   the error band that FP64 reversed (must be 0) */
    int64_t probe_tests[PC_MAX_LEVEL + 1];   /* ordered runs: tests of the probe pass (included in
                                                tests) */
    int64_t probe_removed[PC_MAX_LEVEL + 1]; /* ordered runs: edges the probe pass removed (included
                                                in removed) */
    int32_t max_degree[PC_MAX_LEVEL + 1];/* max degree of G' at the start of the level (0 at level 0) */
    int32_t levels_run;                  /* levels executed, level 0 included */
    int32_t fp64_from;                   /* 0, or the level from which the run was completed in
                                            FP64 because the FP64 re-check queue (recheck_cap)
                                            overflowed there; that level's counts include both of
                                            its passes */
    float prep_ms;                       /* column statistics + standardization (timing & 16) */
    float corr_ms;                       /* correlation GEMM with the level-0 test (timing & 1) */
    float compact_ms[PC_MAX_LEVEL + 1];  /* compaction + planning of level l (timing & 4) */
    float level_ms[PC_MAX_LEVEL + 1];    /* level kernel of level l (timing & 2) */
    float recheck_ms[PC_MAX_LEVEL + 1];  /* FP64 re-check kernel of level l (timing & 8) */
    double wall_ms;                      /* host wall time of the call */
} pc_run_stats;

typedef struct pc_ctx pc_ctx;

/* Creates a context bound to the current HIP device and to `stream` (a hipStream_t; NULL = the
 * null stream). opt may be NULL for defaults. Allocates only small handles. */
pc_status pc_create(pc_ctx **out, void *stream, const pc_options *opt);
void pc_destroy(pc_ctx *ctx);
pc_status pc_default_options(pc_options *opt);

/* Bytes of device workspace pc_corr / pc_level / pc_skeleton need for an n-variable, m-sample
 * problem under opt (NULL = defaults). The workspace holds the standardized data (FP64 copy for
 * re-checks), C, the compacted neighbour lists, the work plan and counters. */
size_t pc_workspace_bytes(int64_t n, int64_t m, const pc_options *opt);

/* Correlation matrix and level 0 (Sec. 3.2, Algorithm 3; at level 0 the CI test of Sec. 4.3 is
 * the Fisher z of C[V_i,V_j] itself against tau_0).
 *   X        device, m x n FP64 row-major, read only.
 *   alpha    significance level in (0, 1).
 *   ws       device workspace of ws_bytes >= pc_workspace_bytes(n, m, opt), 256-byte aligned.
 *   C_out    optional device n x n row-major copy of C (FP64 for PC_PREC_FP64, else FP32); C_aa = 1.
 *   adj_out  optional device bit matrix (layout above): G after level 0.
 * Standardizes the columns (two-pass mean, FP64), forms C = Z^T Z with MFMA, tests every pair
 * i < j at level 0 (|atanh C_ij| <= tau_0 removes it) and leaves C and G in the workspace for
 * pc_level. Errors: PC_ERR_CONSTANT_COLUMN / PC_ERR_NONFINITE are detected on the device and
 * reported by the next synchronising call (pc_level, pc_skeleton, pc_sync_status). */
pc_status pc_corr(pc_ctx *ctx, const double *X, int64_t m, int64_t n, double alpha, void *ws,
                  size_t ws_bytes, void *C_out, uint64_t *adj_out);

/* One level l >= 1 of Algorithm 1 (Sec. 2.4; the body of Algorithm 2 for l >= 1: compact A_G into
 * A'_G, then run the level's CI tests, Sec. 3.3-3.4 and 4.1-4.3).
 *   level    1 <= level <= PC_MAX_LEVEL.
 *   adj      device bit matrix, in/out: G before the level (this becomes the snapshot G'), G after.
 *   sep      SepSet table; one record is appended per removed edge.
 *   st       optional host statistics; fields for `level` are filled.
 *   ws       the workspace of a preceding pc_corr call with the same n, m (C and the FP64
 *            standardized data are read from it).
 * The conditioning sets of edge (i,j) are drawn from adj(i,G')\{j} and from adj(j,G')\{i}; the
 * first independent test removes the edge from G and records S. Runs nothing and returns
 * PC_WARN_SAMPLE_LIMIT if m - level - 3 <= 0. Synchronises the stream. */
pc_status pc_level(pc_ctx *ctx, int level, int64_t n, int64_t m, double alpha, uint64_t *adj,
                   const pc_sepset *sep, pc_run_stats *st, void *ws, size_t ws_bytes);

/* Levels on a correlation matrix the caller supplies instead of data. The CI test of Sec. 4.3
 * (Eq. 3-6) needs only C and the sample size, so these calls take C and a sample size m given as a
 * double: a population correlation matrix with a nominal m such as 1e20 runs the tests in the
 * large-sample limit, where PC-stable returns the skeleton of the true DAG and every SepSet
 * d-separates its pair (Sec. 2.4). FP64 only: the context's precision must be PC_PREC_FP64
 * (PC_ERR_UNSUPPORTED otherwise), since there are no data to re-check FP32 decisions against.
 *   C        device n x n FP64 row-major, symmetric, finite, C_aa = 1; read only (copied into the
 *            workspace). Pair (i,j) is decided on C[min(i,j), max(i,j)].
 *   m        sample size in tau_l = z / sqrt(m - l - 3) (Eq. 6); must be > 0 and finite. A level with
 *            m - l - 3 <= 0 is not run (PC_WARN_SAMPLE_LIMIT), as in pc_level.
 *   ws       device workspace of at least pc_corr_workspace_bytes(n, opt) bytes, 256-byte aligned.
 * pc_level_corr runs one level l >= 1 on the caller's G (in/out, as pc_level); pc_skeleton_corr runs
 * level 0 on C and then the level loop of pc_skeleton (adj_out, sep, st, max_level as there). Both
 * synchronise the stream. */
size_t pc_corr_workspace_bytes(int64_t n, const pc_options *opt);
pc_status pc_level_corr(pc_ctx *ctx, int level, const double *C, int64_t n, double m, double alpha,
                        uint64_t *adj, const pc_sepset *sep, pc_run_stats *st, void *ws, size_t ws_bytes);
pc_status pc_skeleton_corr(pc_ctx *ctx, const double *C, int64_t n, double m, double alpha, int max_level,
                           uint64_t *adj_out, const pc_sepset *sep, pc_run_stats *st, void *ws,
                           size_t ws_bytes);

/* The whole skeleton step (Algorithm 1 / Algorithm 2): pc_corr, then levels 1, 2, ... while the
 * maximum degree of G minus 1 is >= l (and l <= max_level if max_level >= 0). The stop rule is
 * evaluated on the device; the host reads the maximum degree once, after planning level 2, to
 * bound how many levels it enqueues (degrees only shrink, so later levels cannot need more).
 *   X        device m x n FP64 data.
 *   adj_out  device bit matrix: the skeleton.
 *   sep      SepSet table (count is zeroed first).
 *   st       optional host statistics.
 * Synchronises the stream. Returns PC_OK, a warning (the skeleton is what the levels run so far
 * give) or an error. */
pc_status pc_skeleton(pc_ctx *ctx, const double *X, int64_t m, int64_t n, double alpha,
                      int max_level, uint64_t *adj_out, const pc_sepset *sep, pc_run_stats *st,
                      void *ws, size_t ws_bytes);

/* pc_skeleton without a workspace argument, for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid hipMalloc between calls). The workspace is a device array
 * of PC_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on until the process
 * ends; the call itself allocates nothing (no hipMalloc, hipFree or host pinning: the context
 * created those beforehand). Inputs and outputs are the caller's, as for pc_skeleton.
 * Limits: pc_workspace_bytes(n, m, opt) <= PC_NOALLOC_SCRATCH_BYTES (about n = 1000 at m = 500 in
 * FP32) and n <= 8191; larger problems return PC_ERR_WORKSPACE and run nothing.
 * All calls on one GPU share its array, and each call overwrites it (the call clears what must start
 * at zero): calls that overlap in time on the same GPU, from any context or stream, race and give
 * undefined results. Synchronises the stream. */
#define PC_NOALLOC_SCRATCH_BYTES (64u << 20)
pc_status pc_skeleton_noalloc(pc_ctx *ctx, const double *X, int64_t m, int64_t n, double alpha,
                              int max_level, uint64_t *adj_out, const pc_sepset *sep, pc_run_stats *st);

/* One dataset of a batch (Sec. 5 of the paper runs one dataset at a time; a batch runs many
 * independent skeletons together, their work items tagged by dataset).
 *   X        device m x n FP64 row-major data.
 *   alpha    significance level in (0, 1); max_level as for pc_skeleton.
 *   adj_out  device bit matrix (n x ceil(n/64) uint64): the skeleton.
 *   sep      SepSet table of this dataset (count is zeroed by the run). */
typedef struct {
    const double *X;
    int64_t m, n;
    double alpha;
    int32_t max_level;
    int32_t pad;
    uint64_t *adj_out;
    pc_sepset sep;
} pc_problem;

/* Bytes of device workspace for a batch (the same workspace serves pc_batch_skeleton and
 * pc_batch_capture). Returns 0 for an invalid batch. */
size_t pc_batch_workspace_bytes(const pc_problem *probs, int count, const pc_options *opt);

/* Runs the skeletons of `count` independent datasets together: every kernel launch serves all of
 * them (correlation tiles, rows and work items of all datasets share one index space), and the
 * level loop runs on the device until no dataset has work left (or every cap is reached).
 *   probs    host array of count problem descriptors (their buffers are device memory).
 *   st       optional host array of count statistics; status optional host array of count
 *            per-dataset results (PC_OK, a warning, or an error as for pc_skeleton).
 * Synchronises the stream. Returns PC_OK if every dataset succeeded or only warned, else the first
 * error. */
pc_status pc_batch_skeleton(pc_ctx *ctx, const pc_problem *probs, int count, pc_run_stats *st,
                            pc_status *status, void *ws, size_t ws_bytes);

/* A captured batch: the batched skeleton (standardize, correlation, and levels 1 .. G, where G is
 * the smaller of opt.graph_levels and the largest cap of the batch; each kernel exits at once when
 * no work is left) recorded once as a hipGraph and replayed with pc_graph_launch. The graph keeps
 * the pointers it was captured with: new data is run by writing it into the same X buffers. The
 * context's stream must not be the null stream. */
typedef struct pc_graph pc_graph;
pc_status pc_batch_capture(pc_ctx *ctx, const pc_problem *probs, int count, void *ws,
                           size_t ws_bytes, pc_graph **out);
/* Enqueues one replay on the context's stream (asynchronous). */
pc_status pc_graph_launch(pc_graph *g);
/* Waits for the last replay and reports per-dataset statistics and results (as pc_batch_skeleton).
 * If a dataset still has work after the recorded levels, the remaining levels are run on the
 * context's stream first (ordinary launches), so the results are always those of the whole
 * skeleton. */
pc_status pc_graph_results(pc_graph *g, pc_run_stats *st, pc_status *status);
void pc_graph_destroy(pc_graph *g);

/* ---------------------------------------------------------------------------------------------
 * Learned conditioning-set ordering.
 *
 * PC-stable's skeleton does not depend on the order in which conditioning sets are tried (Sec. 2.4),
 * so a level may first test, for every edge (i,j), the subsets of the candidates k in
 * adj(i,G')\{j} that a model ranks highest, then run the plain enumeration on the same G'. The
 * model is an MLP 8 -> 64 -> 64 -> 1 (ReLU) on the candidate features
 *   |C_ij|, |C_ik|, |C_jk|, |rho_ij.k|, d_i/64, d_j/64, d_k/64, level/8
 * (rho_ij.k the level-1 partial correlation, degrees in G'). Parameters are PC_MLP_PARAMS FP32
 * values laid out as W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3 (weights row = output).
 * ------------------------------------------------------------------------------------------- */
#define PC_MLP_IN 8
#define PC_MLP_HID 64
#define PC_MLP_PARAMS 4801

typedef struct {
    const float *params;      /* edge model, device, PC_MLP_PARAMS values (NULL: no probe pass) */
    const float *row_params;  /* shared-set model, device, PC_MLP_PARAMS values (NULL: none) */
    int32_t min_level;    /* first level that runs the probe pass (1..8; default 2) */
    int32_t max_level;    /* last level that runs it (min_level..8; 0 = 8) */
    int32_t top;          /* candidates kept per edge direction (1..8); the probe tests their
                             C(top, level) subsets, so levels above top have no probe */
    int32_t row_top;      /* level 1, shared-set order: the row_top best-scored candidates k of
                             every node are tested first, as sets {k} against all its edges, then
                             the remaining ones (1..16; 0 = off) */
    int32_t row_rank;     /* what ranks the candidates of the shared-set order: 0 = the row model
                             (row_params), 1 = |C_ik| alone (row_params unused, may be NULL) */
    int32_t row_short;    /* row model only: 0 = it scores every candidate of a node; K in
                             row_top..64 = it scores only the K candidates of largest |C_ik| (ties:
                             lower position first), and the row_top chosen come from those */
    int32_t row_sort;     /* 1: the candidates after the row_top chosen are enumerated by
                             descending |C_ik| instead of ascending id (0) */
    int32_t row_split;    /* > row_top: the remaining sets of level 1 run in two level-kernel passes,
                             ranks [row_top, row_split) of every node first, then the rest; 0 = one
                             pass */
} pc_order;

/* Workspace of pc_skeleton_ordered (the probe keeps its features and scores on chip, so this is
 * pc_workspace_bytes). */
size_t pc_ordered_workspace_bytes(int64_t n, int64_t m, const pc_options *opt, const pc_order *order);

/* pc_skeleton with a learned order of the conditioning sets (two forms, either or both):
 *  - shared-set order (row_top, with row_params or row_rank 1): at level 1 every node i of degree
 *    2..1024 ranks its candidates k. k*, the candidate of largest |C_ik|, always comes first; the row
 *    model picks the next row_top - 1 from (i, k) features (|C_ik|, |C_ik| over the row's largest,
 *    the overlap of N_i and N_k against a random graph's, d_k / (d_i + d_k), |C_k k*|,
 *    |rho_ik.k*|, the row mean of |C_ij| over its largest, |N_i & N_k| / d_i), or |C_ik| ranks
 *    them all (row_rank 1). The sets {k} of the row_top chosen are tested against every edge of the
 *    row before the rest of the enumeration (row_sort, row_split: how the rest is ordered and cut);
 *  - probe pass (params): before every level l with min_level <= l <= max_level and l <= top. The probe runs in one kernel per level: for every row i of G' with l + 1 <= d_i <= 48,
 * the MLP (BF16 weights and activations, FP32 accumulation) scores every candidate k of every
 * edge (i, j), and for every live edge the C(top, l) subsets of its best-scored candidates are
 * tested with the level's test (rows with more neighbours are left to the plain enumeration). The
 * adjacency after every level and the skeleton are those of pc_skeleton; SepSets may differ (any
 * separating S is valid). Statistics report the probe's tests and removals separately. */
pc_status pc_skeleton_ordered(pc_ctx *ctx, const double *X, int64_t m, int64_t n, double alpha,
                              int max_level, const pc_order *order, uint64_t *adj_out,
                              const pc_sepset *sep, pc_run_stats *st, void *ws, size_t ws_bytes);

/* pc_batch_capture with a learned conditioning-set order recorded into the graph (the forms and
 * fields of pc_order as for pc_skeleton_ordered; order NULL is pc_batch_capture). The order is
 * copied, but the model parameters it points to are read at every replay: they must stay valid and
 * unchanged while the graph is used. */
pc_status pc_batch_capture_ordered(pc_ctx *ctx, const pc_problem *probs, int count, const pc_order *order,
                                   void *ws, size_t ws_bytes, pc_graph **out);

/* ---------------------------------------------------------------------------------------------
 * Autotuned launch shapes.
 *
 * How fast a level runs depends on how its conditioning sets are cut into work items and staged:
 * the paper tunes its kernels' shapes per dataset (Sec. 5.4, the configuration study). Because
 * the skeleton does not depend on these shapes (nor on the order of work, Sec. 2.4), every level
 * can be timed under each candidate shape on the real workload and take its own best.
 * ------------------------------------------------------------------------------------------- */
typedef struct {
    int32_t tests_per_lane[PC_MAX_LEVEL + 1]; /* item size bound of level l (as pc_options;
                                                 0 = the context's option or rule) */
    int32_t ranks_per_lane[PC_MAX_LEVEL + 1]; /* sets per lane in an item (0 = context's) */
    int32_t lds_budget[PC_MAX_LEVEL + 1];     /* LDS staging budget in bytes (-1 = context's;
                                                 0 = the global-memory gather path) */
    int32_t grid[PC_MAX_LEVEL + 1];           /* work-groups of the level kernels (0 = all that
                                                 fit at once) */
    int32_t recheck_grid[PC_MAX_LEVEL + 1];   /* work-groups of the FP64 re-check (0 = 4 per CU) */
    int32_t set_lanes[PC_MAX_LEVEL + 1];      /* levels 1 and 2 only: fewest lanes that share one
                                                 conditioning set, a power of two in 4 .. 64
                                                 (0 = 4); fewer lanes per set run more of a short
                                                 row's sets at once */
    float level_ms[PC_MAX_LEVEL + 1];         /* pc_tune: best time of level l's test and re-check
                                                 kernels */
    float default_ms[PC_MAX_LEVEL + 1];       /* pc_tune: the same with the context's shapes */
    int32_t levels;                           /* levels 1 .. levels - 1 were timed */
    int32_t runs;                             /* skeleton runs the search took */
} pc_tuning;

/* Measures the level and re-check kernels of the batch `probs` (or, with count = 1 and order
 * non-NULL, of pc_skeleton_ordered on it) under candidate shapes, one parameter at a time for all
 * levels together: tests_per_lane in {16 .. 2048}, lds_budget in {0, 8 KiB, 16 KiB, 32 KiB},
 * ranks_per_lane in {1, 2, 4, 8}, grid in {16, 64, 256} work-groups, recheck_grid in {16, 64, 256}
 * and (levels 1 and 2) set_lanes in {16, 64}.
 * Each level keeps a value at least 1% faster than its current one (HIP events; the faster of two
 * runs), or one within 2% of the fastest time seen at that level that runs at least 10% fewer CI
 * tests than its current one. level_ms is the time of the kept shape. Writes the result to *out and applies it to the context (as pc_set_tuning). Runs the
 * skeleton about 40 times, so the problems' outputs hold a complete, correct result afterwards; ws
 * as for pc_batch_skeleton (or pc_skeleton_ordered). Returns the first error of a run, or
 * PC_ERR_INVALID_ARG (order with count > 1). */
pc_status pc_tune(pc_ctx *ctx, const pc_problem *probs, int count, const pc_order *order, void *ws,
                  size_t ws_bytes, pc_tuning *out);
/* Applies per-level shapes to later launches on ctx (graphs capture them as they are when
 * captured); NULL returns to the context's options. A copy is kept. Values out of range are
 * PC_ERR_INVALID_ARG. */
pc_status pc_set_tuning(pc_ctx *ctx, const pc_tuning *t);

/* Candidate features of level `level` for the snapshot adj (device bit matrix, not modified), for
 * training data: rows ordered by i, then j = N_i[p], then k in N_i\{j}, as the ordered run uses them.
 *   feats    device rows x 8 FP32; meta device rows x 3 int32 (i, j, k); cap = rows they hold.
 *   rows_out host: number of rows (returned even when it exceeds cap, with PC_ERR_WORKSPACE).
 *   ws       workspace of a preceding pc_corr on the same data. Synchronises the stream. */
pc_status pc_features(pc_ctx *ctx, int level, int64_t n, int64_t m, double alpha, const uint64_t *adj,
                      float *feats, int32_t *meta, int64_t cap, int64_t *rows_out, void *ws,
                      size_t ws_bytes);

/* Training rows of the shared-set order at level 1 for the snapshot adj (device bit matrix, not
 * modified): one row per (i, k in N_i), ordered by i then position of k, with the 8 features of
 * pc_skeleton_ordered's row model, as label the fraction of the other edges (i, j) of the row that
 * {k} separates by the FP32 test (|rho_ij.k| <= tanh(tau_1), no re-check band), and meta (i, k).
 *   feats device rows x 8 FP32; labels device rows FP32; meta device rows x 2 int32 (optional).
 *   level must be 1; other arguments as in pc_features. Synchronises the stream. */
pc_status pc_row_features(pc_ctx *ctx, int level, int64_t n, int64_t m, double alpha, const uint64_t *adj,
                          float *feats, float *labels, int32_t *meta, int64_t cap, int64_t *rows_out,
                          void *ws, size_t ws_bytes);

/* The ranking step of the shared-set order alone, for checking the scoring kernel: for the
 * level-1 snapshot adj (device bit matrix, not modified) it scores the candidates of every node as
 * pc_skeleton_ordered does (order: row_params / row_rank / row_short / row_top) and runs no test.
 *   scores  device n x n FP32: scores[i*n + k] = score of candidate k of node i (the model's BF16
 *           MLP output, or |C_ik| for row_rank 1; -inf outside the short list). Entries of
 *           non-neighbours, and rows that are not ranked (degree < 2 or > 1024), are not written.
 *   top     device n x row_top int32: the chosen candidates of node i, best first (ties: lower
 *           position in the ascending neighbour list); -1 past the node's degree. Rows of degree
 *           < 2 are not written.
 *   ws      workspace of a preceding pc_corr on the same data. Synchronises the stream. */
pc_status pc_row_scores(pc_ctx *ctx, int64_t n, int64_t m, double alpha, const uint64_t *adj, const pc_order *order,
                        float *scores, int32_t *top, void *ws, size_t ws_bytes);

/* MLP kernels (stream ordered, asynchronous), exported for training and gradient checks.
 *   forward : scores[r] = MLP(X[r]) for rows x 8 inputs; act (optional, rows x 128) keeps the
 *             hidden activations for backward.
 *   backward: grads = d(sum_r dscore[r] * score[r]) / d(params); partial is device scratch of
 *             ceil(rows/64) * PC_MLP_PARAMS floats (the per-tile sums, added in a fixed order).
 *   bce     : loss = mean_r [w y softplus(-s) + (1-y) softplus(s)] (device double) and
 *             dscore = dloss/ds.
 *   adam    : one Adam step (step counts from 1) on params with moment buffers m1, m2. */
pc_status pc_mlp_forward(pc_ctx *ctx, const float *params, const float *X, int64_t rows, float *scores,
                         float *act);
pc_status pc_mlp_backward(pc_ctx *ctx, const float *params, const float *X, int64_t rows, const float *act,
                          const float *dscore, float *grads, float *partial);
pc_status pc_mlp_bce(pc_ctx *ctx, const float *scores, const float *labels, int64_t rows, float pos_weight,
                     float *dscore, double *loss);
pc_status pc_mlp_adam(pc_ctx *ctx, float *params, const float *grads, float *m1, float *m2, int step,
                      float lr, float beta1, float beta2, float eps);

/* Orientation of a skeleton into a CPDAG: the step of the PC algorithm after the skeleton
 * (Sec. 2.4), here on the GPU. Unshielded colliders i -> k <- j wherever k is not in SepSet(i, j),
 * then Meek's rules R1-R3 in synchronous rounds until nothing changes. Conventions that make the
 * result independent of the order of work: colliders are judged on the skeleton and SepSets
 * alone, and an edge that receives arrowheads at both ends is bidirected; a round orients every
 * undirected edge that a rule orients in the state at the start of the round, and an edge
 * proposed both ways in the same round stays undirected.
 *   adj     device n x ceil(n/64) u64 skeleton (symmetric, zero diagonal), not modified.
 *   recs    device SepSet records of the level >= 1 removals (as pc_skeleton writes them), nrec of
 *           them; a non-adjacent pair without a record has the empty SepSet (level 0). Records
 *           with ids or levels out of range are ignored.
 *   arrows  device n x ceil(n/64) u64, written: bit y of row x set iff the edge x - y has an
 *           arrowhead at y (x -> y, or x <-> y when row y has bit x too).
 *   ws      workspace of pc_orient_workspace_bytes(n) bytes, 256-byte aligned.
 *   rounds  host (optional): propagation rounds that oriented at least one edge.
 * Synchronises the stream once per round. */
size_t pc_orient_workspace_bytes(int64_t n);
pc_status pc_orient(pc_ctx *ctx, int64_t n, const uint64_t *adj, const pc_sep_rec *recs, int64_t nrec,
                    uint64_t *arrows, void *ws, size_t ws_bytes, int32_t *rounds);

/* Waits for the context's stream and reports device-detected input errors of pc_corr. */
pc_status pc_sync_status(pc_ctx *ctx, void *ws, size_t ws_bytes);

/* Host-only helper, no GPU needed: the t-th (0-based) l-subset of positions {0..d-1} in
 * lexicographic order, the combination function of Sec. 4.2 (Algorithm 6, with the 0-based shift).
 * If skip >= 0 it is the edge form of cuPC-E: the subset is drawn from the d-1 positions other
 * than `skip` (t < C(d-1,l)) and positions >= skip are shifted by one. Writes l ints to out.
 * Returns PC_ERR_INVALID_ARG if t is out of range. */
pc_status pc_comb_unrank(int32_t d, int32_t l, uint64_t t, int32_t skip, int32_t *out);

/* Host-only helper: z = Phi^-1(1 - alpha/2) and tau_l = z / sqrt(m - l - 3) (Eq. 6); returns NaN
 * for tau when m - l - 3 <= 0. */
double pc_threshold(double alpha, double m, int level);

/* Host-only helper: sizeof of the ABI structs, so bindings can check their layouts.
 * which: 0 pc_options, 1 pc_sep_rec, 2 pc_sepset, 3 pc_run_stats, 4 pc_problem, 5 pc_order,
 * 6 pc_tuning; other values return 0. */
size_t pc_abi_size(int which);

/* Text of a status code (static storage). */
const char *pc_status_str(pc_status s);

#ifdef __cplusplus
}
#endif
#endif
