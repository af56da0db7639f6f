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
 * after level PC_MAX_LEVEL and returns PC_WARN_LEVEL_CAP. */
#define PC_MAX_LEVEL 13

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
                                  (default 65536; 0 forces the global-memory gather path) */
    int32_t ranks_per_lane;    /* conditioning sets per lane in one work item (0 = automatic) */
    int32_t grid;              /* work-groups of the persistent level kernel (0 = automatic) */
    int32_t timing;            /* 1: time phases with HIP events into pc_run_stats */
    int64_t recheck_cap;       /* capacity of the FP64 re-check queue in tests per level
                                  (0 = 1<<20); a level that needs more returns PC_ERR_WORKSPACE */
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
    int32_t max_degree[PC_MAX_LEVEL + 1];/* max degree of G' at the start of the level (0 at level 0) */
    int32_t levels_run;                  /* levels executed, level 0 included */
    int32_t pad;
    float corr_ms;                       /* standardize + correlation + level 0 (timing = 1) */
    float compact_ms[PC_MAX_LEVEL + 1];  /* compaction + planning of level l (timing = 1) */
    float level_ms[PC_MAX_LEVEL + 1];    /* level kernel of level l (timing = 1) */
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

/* The whole skeleton step (Algorithm 1 / Algorithm 2): pc_corr, then levels 1, 2, ... while the
 * maximum degree of G minus 1 is >= l (and l <= max_level if max_level >= 0).
 *   X        device m x n FP64 data.
 *   adj_out  device bit matrix: the skeleton.
 *   sep      SepSet table (count is zeroed first).
 *   st       optional host statistics.
 * Synchronises the stream. Returns PC_OK, a warning (the skeleton is what the levels run so far
 * give) or an error. */
pc_status pc_skeleton(pc_ctx *ctx, const double *X, int64_t m, int64_t n, double alpha,
                      int max_level, uint64_t *adj_out, const pc_sepset *sep, pc_run_stats *st,
                      void *ws, size_t ws_bytes);

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
 * which: 0 pc_options, 1 pc_sep_rec, 2 pc_sepset, 3 pc_run_stats; other values return 0. */
size_t pc_abi_size(int which);

/* Text of a status code (static storage). */
const char *pc_status_str(pc_status s);

#ifdef __cplusplus
}
#endif
#endif
