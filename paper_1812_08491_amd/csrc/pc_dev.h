// Library-internal declarations shared by the HIP translation units of libpc.so.
//
// Every kernel works on a batch of independent problems (datasets) described by a device table of
// Prob records; a single-problem call is a batch of one. Work of all problems is flattened into
// one index space per kernel (columns, tiles, rows, work items), so one launch serves the batch.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "pc.h"

namespace pcg {

constexpr int kLevels = PC_MAX_LEVEL + 2;             // per-level arrays: levels 0 .. PC_MAX_LEVEL+1
constexpr int kBinomCols = PC_MAX_LEVEL + 2;          // C(a, b) for b = 0 .. PC_MAX_LEVEL + 1
constexpr unsigned long long kSat = 1ull << 62;       // saturation value of the binomial table
constexpr int kLevelThreads = 256;                    // threads of a level work-group
constexpr int kGramLd = PC_MAX_LEVEL + 2;             // leading dimension of an FP64 Gram block
constexpr int kFastLevels = 13;    // levels whose per-set factor lives in registers (k_level);
                                   // deeper levels factor each set across a wavefront
constexpr int kWaveSetLevels = 2;  // levels whose conditioning sets are shared by a group of lanes
                                   // (up to a whole wavefront) that divide the set's candidates

// 64-bit signed counter add (two's complement, so the unsigned atomic is exact).
__device__ inline void add_ll(long long *p, long long v) {
    atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v);
}

// Exclusive prefix sum of v over the kThreads threads of a work-group (kThreads a multiple of 64,
// at most 4096): a shuffle scan inside each wavefront, then one over the wavefront totals. total
// receives the sum over all threads. lds: kThreads / 64 slots, free again after the next barrier.
template <int kThreads>
__device__ inline long long block_exclusive_scan(long long v, long long *lds, long long &total) {
    static_assert(kThreads % 64 == 0 && kThreads <= 64 * 64, "work-group size");
    constexpr int kWaves = kThreads / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    long long incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) lds[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        long long w = lane < kWaves ? lds[lane] : 0;
#pragma unroll
        for (int o = 1; o < kWaves; o <<= 1) {
            const long long t = __shfl_up(w, o, 64);
            if (lane >= o) w += t;
        }
        if (lane < kWaves) lds[lane] = w;
    }
    __syncthreads();
    total = lds[kWaves - 1];
    return (wave > 0 ? lds[wave - 1] : 0) + incl - v;
}

// One problem of a batch: shapes, buffers (device pointers), thresholds and statistics.
struct Prob {
    int64_t n, m, mp, W;
    const double *X;               // m x n FP64 row-major input
    double *mu, *inv;              // column mean and 1 / ||X - mu||
    double *zt64;                  // n x mp FP64 standardized data (variable-major)
    void *zlo, *zhi;               // low-precision GEMM operands
    void *C;                       // n x n correlation (FP64 or FP32)
    unsigned long long *adj;       // live G (bit matrix)
    int *nbr, *deg;                // compacted G' (row i at nbr + i*n), degrees
    pc_sep_rec *recs;
    long long rec_cap;
    long long *rec_count;
    int max_level;                 // last level to run (PC_MAX_LEVEL + 1: until the stop rule)
    int err;                       // device-detected input error (pc_status)
    int tail_next;                 // after the tail kernel: level it left to the level kernels (0: none)
    int tail_done;                 // levels up to this one were run (or found empty) by the tail kernel
    double t0, eps_c;              // level 0: tanh(tau_0) and the C error bound (low precision)
    double tau[kLevels];           // tau_l; NaN when m - l - 3 <= 0
    float t[kLevels];              // tanh(tau_l) in FP32
    float band[kLevels];           // FP32 error band scale of level l
    long long tests[kLevels], removed[kLevels], rechecks[kLevels], items[kLevels];
    long long audit_viol[kLevels];
    long long probe_tests[kLevels], probe_removed[kLevels];
    int maxdeg[kLevels];
};

// The re-check queue is cut into kRqSlices slices with a counter each; a work-group pushes to the
// slice of its index, so the pushes of a level (millions on the BF16x3 path) do not all serialise
// on one address.
constexpr int kRqSlices = 16;

// Device-resident queue state of the current level (one per batch).
struct DevState {
    unsigned long long total_items;  // work items planned for the current level
    unsigned long long next_item;    // queue head (atomic)
    unsigned long long rq_slice[kRqSlices];   // entries pushed to each re-check queue slice this level
    int done;                        // 1 once a planning pass found no work in any problem
    int overflow;                    // a row's subset count exceeded the supported range
    int rq_overflow;                 // 0, or the level whose re-check queue filled up (the level loop
                                     // then stops: done is set)
    int rq_overflow_tail;            // a problem's share of the queue filled up in the tail kernel
    int pad[2];
    unsigned long long item_stride;  // queue order: pop g takes item (g * item_stride) mod total_items
};
static_assert(sizeof(DevState) <= 64 * sizeof(int), "the re-arm kernel clears DevState with 64 threads");


// Re-check queue entry: a test whose FP32 decision fell in the error band (or, on the FP64 path,
// whose M2 is rank deficient).
struct RqEntry {
    int prob, i, j, cls;           // cls: FP32 class (0 dependent, 1 independent, 2 in the band)
    uint16_t S[PC_MAX_LEVEL];      // variable ids (n <= 65536)
    uint16_t pad[(8 - PC_MAX_LEVEL % 8) % 8];
};
static_assert(sizeof(RqEntry) % 16 == 0, "queue entries stay 16-byte aligned");

// Flattened index tables and shared buffers of a batch (passed by value to every kernel).
struct Batch {
    Prob *probs;
    int count;
    int prec;
    int force_recheck;
    int lane_tests;                // bound on the CI tests one lane runs per work item (0: none)
    int set_lanes;                 // level 1: fewest lanes that share one conditioning set
    const long long *row_base;     // count + 1: first flattened row of each problem
    const long long *cs_base;      // count + 1: first k_colstats block
    const long long *st_base;      // count + 1: first k_standardize block
    const long long *tile_base;    // count + 1: first k_corr tile
    long long *nitems;             // per flattened row: work items of the level
    long long *item_off;           // total_rows + 1 exclusive offsets
    int *rowdeg;                   // per flattened row: its degree in G' and its problem (2 x
                                   // total_rows ints, written by the compaction for the planner)
    const unsigned long long *binom;
    DevState *st;
    RqEntry *rq;
    long long rq_cap;
    long long total_rows;
    // Conditioning-set ranks a level launch covers: [rank_lo, rank_hi) of each row's lexicographic
    // enumeration (0 and ~0 for all of them); probe = 1 marks the probe pass of a learned order,
    // whose tests and removals are also counted as probe statistics.
    unsigned long long rank_lo, rank_hi;
    int probe;
    // Level 1 after the shared-set order with sorted enumeration: a row of G' that the order
    // ranked (l1_ranked below) keeps its ascending neighbour list, and its set ranks t map to list
    // positions through the permutation stored after the list, nbr[i*n + d + t].
    int l1_perm;
    int corr_only;    // the correlation kernel writes C only (no level-0 test, no adjacency)
};


// The re-check entries of a level: slice s holds min(rq_slice[s], cap_s) entries from index
// s * cap_s on, cap_s = rq_cap / kRqSlices. Entries are numbered 0 .. total() - 1 across slices.
struct RqView {
    long long cap_s;
    long long start[kRqSlices + 1];
    __device__ explicit RqView(const Batch &b) {
        cap_s = b.rq_cap / kRqSlices;
        start[0] = 0;
        for (int s = 0; s < kRqSlices; ++s) {
            const unsigned long long c = b.st->rq_slice[s];
            start[s + 1] = start[s] + (c < (unsigned long long)cap_s ? (long long)c : cap_s);
        }
    }
    __device__ long long total() const { return start[kRqSlices]; }
    __device__ long long index(long long e) const {   // queue position of entry e
        int s = 0;
        while (s + 1 < kRqSlices && start[s + 1] <= e) ++s;
        return (long long)s * cap_s + (e - start[s]);
    }
};

// Rows the level-1 shared-set order ranks: degree up to kRowOrderCap and at most kRowOrderWords
// adjacency words (both staged in LDS by the ordering kernel).
constexpr int kRowOrderCap = 512;
constexpr int kRowOrderWords = 256;
__host__ __device__ inline bool l1_ranked(int64_t d, int64_t W) { return d <= kRowOrderCap && W <= kRowOrderWords; }
// The rank permutation fits after the neighbour list of a row of degree d when 2 d <= n.
__host__ __device__ inline bool l1_perm_row(const Batch &b, int64_t d, int64_t W, int64_t n) {
    return b.l1_perm && l1_ranked(d, W) && 2 * d <= n;
}

// The ranks [lo, hi) of a row with nS conditioning sets that a launch covers.
__host__ __device__ inline void rank_window(const Batch &b, unsigned long long nS, unsigned long long &lo,
                                            unsigned long long &hi) {
    lo = b.rank_lo < nS ? b.rank_lo : nS;
    hi = b.rank_hi < nS ? b.rank_hi : nS;
}

// Conditioning sets per work item of a row of degree d at level l, from the base count R. A set
// costs about d - l tests (one per j), so rows with long neighbour lists get fewer sets per item,
// down to one set whose j loop the whole work-group splits, until a lane runs at most `lane_tests`
// tests per item. Deep levels (one set per wavefront) keep R. The planner and the level kernel
// call this with the same arguments, so they agree on the item layout of every row.
__host__ __device__ inline long long item_sets(int d, int l, long long R, int lane_tests) {
    if (lane_tests <= 0 || l > kFastLevels) return R;
    const long long jn = d - l > 1 ? d - l : 1;
    long long r = R;
    while (r > 1 && r * jn > (long long)lane_tests * kLevelThreads) r >>= 1;
    return r;
}

// Largest k in [0, count) with base[k] <= x (base ascending, base[0] = 0).
__device__ inline int find_base(const long long *base, int count, long long x) {
    int lo = 0, hi = count;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (base[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

inline int64_t pad_m(int64_t m) { return (m + 63) / 64 * 64; }
inline int64_t words_per_row(int64_t n) { return (n + 63) / 64; }
inline size_t align256(size_t x) { return (x + 255) / 256 * 256; }

constexpr int kCsCols = 16;        // columns per k_colstats block
inline int64_t cs_blocks(int64_t n) { return (n + kCsCols - 1) / kCsCols; }
inline int64_t st_blocks(int64_t n, int64_t mp) { return ((n + 63) / 64) * (mp / 64); }
inline int64_t corr_tiles(int64_t n) { const int64_t T = (n + 63) / 64; return T * (T + 1) / 2; }

// ---- launchers (each translation unit launches only its own kernels) ----

// pc_prep.hip
hipError_t launch_binom(hipStream_t s, unsigned long long *binom, int64_t rows);
hipError_t launch_init(hipStream_t s, const Batch &b);
hipError_t launch_rearm(hipStream_t s, const Batch &b);
hipError_t launch_colstats(hipStream_t s, const Batch &b, long long blocks);
hipError_t launch_standardize(hipStream_t s, const Batch &b, long long blocks);

// pc_corr.hip
hipError_t launch_corr(hipStream_t s, const Batch &b, long long tiles, int num_cu);
hipError_t launch_level0_given(hipStream_t s, const Batch &b);

// pc_level.hip
hipError_t launch_compact(hipStream_t s, const Batch &b, int level, int ranks_per_item);
hipError_t launch_plan(hipStream_t s, const Batch &b, int level);
// Work items of a rank window over the current G' (no compaction), then its queue; the level's
// stop flag, statistics and re-check queue are left as they are.
hipError_t launch_window(hipStream_t s, const Batch &b, int level, int ranks_per_item);
hipError_t launch_level(hipStream_t s, const Batch &b, int level, int ranks_per_item, int lds_bytes,
                        int grid);
hipError_t launch_recheck(hipStream_t s, const Batch &b, int level, int grid);
int recheck_blocks_per_cu();                                    // resident re-check work-groups per CU

// pc_orient.hip
// Skeleton orientation: clears the state, indexes the SepSet records, marks the unshielded
// colliders (OUT / IN: n x W arrowhead bit matrices; P0, P1: proposal buffers; sep_idx: n x n).
hipError_t launch_orient_setup(hipStream_t s, int64_t n, const unsigned long long *A, const pc_sep_rec *recs,
                               int64_t nrec, unsigned long long *OUT, unsigned long long *IN,
                               unsigned long long *P0, unsigned long long *P1, int *sep_idx, int *flag);
// One propagation round: proposals into P (cleared before), applied; Q cleared for the next round;
// *flag = number of edges oriented.
hipError_t launch_orient_round(hipStream_t s, int64_t n, const unsigned long long *A, unsigned long long *OUT,
                               unsigned long long *IN, unsigned long long *P, unsigned long long *Q, int *flag);

// pc_tail.hip
// The remaining levels from `level` of every problem, one work-group per problem, as long as a
// level has at most cap_tests CI tests (an upper bound from the degrees) and l <= kFastLevels.
hipError_t launch_tail(hipStream_t s, const Batch &b, int level, long long cap_tests);
int level_blocks_per_cu(int prec, int level, int lds_bytes);   // resident work-groups per CU
size_t level_lds_fixed(int prec);

// pc_mlp.hip
hipError_t launch_mlp_forward(hipStream_t s, const float *params, const float *X, long long rows,
                              const long long *rows_dev, long long rows_cap, float *scores, float *act,
                              const int *skip, int grid);
hipError_t launch_mlp_backward(hipStream_t s, const float *params, const float *X, long long rows,
                               const float *act, const float *dscore, float *partial, float *grads);
hipError_t launch_bce(hipStream_t s, const float *scores, const float *labels, long long rows, float pos_weight,
                      float *dscore, double *loss);
hipError_t launch_adam(hipStream_t s, float *params, const float *grads, float *m1, float *m2, int step, float lr,
                       float beta1, float beta2, float eps);
hipError_t launch_feat_plan(hipStream_t s, const Batch &b, long long *foff, long long cap, int *skip);
hipError_t launch_features(hipStream_t s, const Batch &b, int level, const long long *foff, float *feats,
                           int *meta, const int *skip);
// Shared-set order: reorders each row's neighbour list, the `top` best-scored candidates first, and
// tests their sets. grid: compute units (the launch fills them).
hipError_t launch_row_order(hipStream_t s, const Batch &b, int level, const float *params, int top, int by_abs,
                            int short_k, int sort_rest, int grid, float *scores_out = nullptr,
                            int *top_out = nullptr);
// Training rows of the shared-set order (features, labels, meta (i, k)) after a compaction.
hipError_t launch_row_features(hipStream_t s, const Batch &b, int level, long long *foff, long long cap, int *skip,
                               float *feats, float *labels, int *meta);
// grid: compute units; the probe launches as many work-groups per unit as fit.
hipError_t launch_probe(hipStream_t s, const Batch &b, int level, const float *params, int topq, int grid);

}  // namespace pcg
