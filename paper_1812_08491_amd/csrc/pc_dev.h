// Library-internal declarations shared by the HIP translation units of libpc.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "pc.h"

namespace pcg {

// Device-resident run state: the work queue of the current level, the stop flag that replaces the
// host-side max-degree test of Algorithm 2, and per-level counters.
struct DevState {
    unsigned long long total_items;  // work items planned for the current level
    unsigned long long next_item;    // queue head (atomic)
    unsigned long long total_sets;   // sum over rows of C(d_i, l)
    int max_deg;                     // max degree of G' found by the last compaction
    int done;                        // 1 once a compaction found no row with d_i >= l + 1
    unsigned int blocks_done;        // finished-block counter of the compaction kernel
    int err;                         // device-detected input error (pc_status), 0 = none
    int deg_work;                    // atomicMax scratch of the compaction kernel
    int overflow;                    // a row's subset count exceeded the supported range
    int rq_overflow;                 // the re-check queue filled up
    int pad;
    unsigned long long rq_count;     // entries pushed to the re-check queue this level
    long long tests[PC_MAX_LEVEL + 2];
    long long removed[PC_MAX_LEVEL + 2];
    long long rechecks[PC_MAX_LEVEL + 2];
    long long items[PC_MAX_LEVEL + 2];
    long long audit_viol[PC_MAX_LEVEL + 2];  // audit mode: FP32 decisions outside the band that
                                             // disagree with FP64
    int maxdeg[PC_MAX_LEVEL + 2];
};

// 64-bit signed counter add (two's complement, so the unsigned atomic is exact).
__device__ inline void add_ll(long long *p, long long v) {
    atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v);
}

constexpr int kBinomCols = PC_MAX_LEVEL + 2;          // C(a, b) for b = 0 .. PC_MAX_LEVEL + 1
constexpr unsigned long long kSat = 1ull << 62;       // saturation value of the binomial table
constexpr int kLevelThreads = 256;                    // threads of a level work-group
constexpr int kGramLd = PC_MAX_LEVEL + 2;             // leading dimension of a per-wave FP64 Gram

inline int64_t pad_m(int64_t m) { return (m + 63) / 64 * 64; }
inline int64_t words_per_row(int64_t n) { return (n + 63) / 64; }
inline size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Workspace layout (byte offsets from the workspace base).
struct Layout {
    int64_t n, m, mp;
    int prec;
    size_t state, mu, inv, zt64, zlo, zhi, c, adj, nbr, deg, nitems, item_off, binom, rq, total;
    int64_t rq_cap;

    static Layout make(int64_t n, int64_t m, int prec, int64_t rq_cap) {
        Layout L{};
        L.n = n;
        L.m = m;
        L.mp = pad_m(m);
        L.prec = prec;
        size_t o = 0;
        auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
        L.state = take(sizeof(DevState));
        L.mu = take(sizeof(double) * n);
        L.inv = take(sizeof(double) * n);
        L.zt64 = take(sizeof(double) * n * L.mp);
        // FP32 mode: zlo holds the FP32 copy; BF16x3 mode: zhi and zlo hold the two BF16 halves.
        size_t low_bytes = prec == PC_PREC_FP32 ? sizeof(float) * n * L.mp
                         : prec == PC_PREC_BF16X3 ? sizeof(uint16_t) * n * L.mp : 0;
        L.zlo = take(low_bytes);
        L.zhi = take(prec == PC_PREC_BF16X3 ? sizeof(uint16_t) * n * L.mp : 0);
        L.c = take((prec == PC_PREC_FP64 ? sizeof(double) : sizeof(float)) * n * n);
        L.adj = take(sizeof(unsigned long long) * n * words_per_row(n));
        L.nbr = take(sizeof(int32_t) * n * n);
        L.deg = take(sizeof(int32_t) * n);
        L.nitems = take(sizeof(long long) * n);
        L.item_off = take(sizeof(long long) * (n + 1));
        L.binom = take(sizeof(unsigned long long) * (n + 1) * kBinomCols);
        L.rq_cap = rq_cap;
        L.rq = take(sizeof(pc_sep_rec) * rq_cap);
        L.total = o;
        return L;
    }
};

// ---- launchers (each translation unit launches only its own kernels) ----

// pc_prep.hip
hipError_t launch_init(hipStream_t s, DevState *st, unsigned long long *binom, int64_t n,
                       long long *zero_me);
hipError_t launch_rearm(hipStream_t s, DevState *st);
hipError_t launch_colstats(hipStream_t s, const double *X, int64_t m, int64_t n, double *mu,
                           double *inv, DevState *st);
hipError_t launch_standardize(hipStream_t s, const double *X, int64_t m, int64_t n, int64_t mp,
                              const double *mu, const double *inv, double *zt64, void *zlo,
                              void *zhi, int prec);

// pc_corr.hip
struct CorrArgs {
    const double *zt64;
    const void *za;        // FP32 copy (FP32 mode) or BF16 high half (BF16x3 mode)
    const void *zb;        // BF16 low half (BF16x3 mode)
    void *C;               // n x n, FP64 or FP32
    unsigned long long *adj;
    DevState *st;
    int64_t n, m, mp, W;
    double tau0;           // level-0 threshold on the Fisher z
    double t0;             // tanh(tau0): threshold on |r|
    double eps_c;          // bound on |C_low - C_fp64| for the FP32 / BF16x3 paths
    int force_recheck;
};
hipError_t launch_corr(hipStream_t s, const CorrArgs &a, int prec);

// pc_level.hip
struct LevelArgs {
    const void *C;                 // n x n FP32 or FP64
    const double *zt64;            // n x mp FP64 standardized data (FP32 paths' re-checks)
    unsigned long long *adj;       // live G (bit matrix)
    const int *nbr;                // compacted G': row i at nbr + i*n
    const int *deg;
    const long long *item_off;     // n + 1 exclusive offsets of work items per row
    const unsigned long long *binom;
    DevState *st;
    pc_sep_rec *recs;
    long long *rec_count;
    long long rec_cap;
    int64_t n, m, mp, W;
    int level;
    int ranks_per_item;            // conditioning sets per work item
    int lds_bytes;                 // dynamic LDS per work-group
    int force_recheck;
    double tau;                    // level threshold on the Fisher z (FP64 decisions)
    float t;                       // tanh(tau) (FP32 decisions)
    float band;                    // margin_scale * (eps_c + rounding) for the FP32 band
    pc_sep_rec *rq;                // re-check queue (level field = FP32 class: 0 dep, 1 indep,
                                   // 2 in the band)
    long long rq_cap;
};
struct RecheckArgs {
    const double *zt64;            // FP64 standardized data (NULL: take the block from C64)
    const double *C64;             // FP64 correlation (FP64 precision path)
    unsigned long long *adj;
    DevState *st;
    const pc_sep_rec *rq;
    long long rq_cap;
    pc_sep_rec *recs;
    long long *rec_count;
    long long rec_cap;
    int64_t n, m, mp, W;
    int level;
    int audit;                     // compare FP32 classes with FP64 decisions
    double tau;
};
hipError_t launch_recheck(hipStream_t s, const RecheckArgs &a, int grid);
size_t level_lds_fixed(int prec);
hipError_t launch_compact(hipStream_t s, const unsigned long long *adj, int64_t n, int64_t W,
                          int level, int ranks_per_item, int *nbr, int *deg, long long *nitems,
                          long long *item_off, const unsigned long long *binom, DevState *st);
hipError_t launch_level(hipStream_t s, const LevelArgs &a, int prec, int grid);

}  // namespace pcg
