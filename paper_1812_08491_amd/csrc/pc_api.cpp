// C ABI of libpc.so: argument checks, workspace planning and the level loop (Algorithm 2).
//
// Every call builds a table of problems (one for pc_corr / pc_level / pc_skeleton, many for the
// batch calls), uploads it into the workspace, and enqueues the kernels of pc_prep.hip,
// pc_corr.hip and pc_level.hip. The level loop needs no host decision between levels: a planning
// pass that finds no work sets a device flag and every later kernel exits at once, so a whole
// skeleton is one stream of launches (and can be captured as one hipGraph).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "pc.h"
#include "pc_comb.h"
#include "pc_dev.h"

using namespace pcg;

struct pc_ctx {
    hipStream_t stream;
    pc_options opt;
    int device;
    int num_cu;
    unsigned long long *binom;      // device binomial table, binom_rows x kBinomCols
    int64_t binom_rows;
    void *staging;                  // pinned host staging of problem tables
    size_t staging_bytes;
    hipEvent_t staging_done;        // recorded after each upload; waited on before reuse
    bool staging_pending;
    // Event pairs of the timed phases: prep, corr, and per level compact / level / re-check.
    hipEvent_t ev_prep[2], ev_corr[2];
    hipEvent_t ev_compact[kLevels][2], ev_level[kLevels][2], ev_recheck[kLevels][2];
    int top_run;                    // highest level enqueued by the current call
    int level_grid[kLevels];        // work-groups of the level kernels: all that fit at once
    int recheck_grid;               // work-groups of the re-check kernel: at most 4 per CU, all resident
    bool tail_enqueued;             // the last enqueue_skeletons ended its levels with the tail kernel
    void *scratch;                  // this device's address of the no-allocation workspace array
    bool tuned;                     // per-level shapes of pc_set_tuning / pc_tune apply
    pc_tuning tuning;
    // Phases whose events the current call recorded (bit l: level l), so that only those are read
    // back: a level the tail kernel ran has none, and events of an earlier call are stale.
    unsigned long long rec_compact, rec_level, rec_recheck;
    bool rec_prep, rec_corr;
};

struct pc_graph {
    pc_ctx *ctx;
    hipGraph_t graph;
    hipGraphExec_t exec;
    unsigned char *ws;
    int count;
    size_t table_off, st_off;
    std::vector<Prob> host_probs;
    std::vector<pc_problem> probs;  // descriptors it was captured with (for continuation)
    int captured;                   // levels recorded in the graph
    int top;                        // last level any dataset may need (PC_MAX_LEVEL + 1 = planning)
    bool tail;                      // the graph ends with the tail kernel (from level captured + 1)
    bool has_order;                 // a learned order was recorded (kept for the continuation)
    pc_order order;
};

// Workspace of pc_skeleton_noalloc: a static device array, one copy per GPU, held until the process
// ends. In host code its name is only a stand-in: kernels and copies use the device address that
// hipGetSymbolAddress returns for the current device (resolved once per device in pc_create).
static __device__ __align__(256) unsigned char scratch[PC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

// This device's address of `scratch` (the device must be current); resolved once per device.
pc_status scratch_address(int dev, void **out) {
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    if (dev < 0 || dev >= kMaxDevices) return PC_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PC_ERR_HIP;
        addr[dev] = p;
    }
    *out = addr[dev];
    return PC_OK;
}

constexpr double kU32 = 5.9604644775390625e-08;  // 2^-24, unit roundoff of FP32
// Default bound on the CI tests of a lane per work item. When every row can have a work-group of
// its own, a level's launch lasts as long as its heaviest row, so heavy rows are cut finer; when
// rows outnumber the work-groups (large problems, batches), the queue balances them, and finer
// items only repeat the row staging.
constexpr int kAutoLaneTests = 128;
constexpr int kAutoLaneTestsSmall = 32;             // when the call has no more rows than work-groups

#define PC_HIP(call)                                                       \
    do {                                                                   \
        hipError_t e_ = (call);                                            \
        if (e_ != hipSuccess) return PC_ERR_HIP;                           \
    } while (0)

pc_options defaults() {
    pc_options o;
    std::memset(&o, 0, sizeof(o));
    o.precision = PC_PREC_FP32;
    o.max_level = -1;
    o.margin_scale = 2.0f;
    o.force_recheck_all = 0;
    o.lds_budget = 16384;
    o.ranks_per_lane = 0;
    o.grid = 0;
    o.timing = 0;
    o.recheck_cap = 0;
    o.graph_levels = 0;
    o.tail_tests = 0;
    return o;
}

bool valid_options(const pc_options &o) {
    if (o.precision < PC_PREC_FP64 || o.precision > PC_PREC_BF16X3) return false;
    if (!(o.margin_scale >= 1.0f)) return false;
    if (o.lds_budget < 0 || o.ranks_per_lane < 0 || o.grid < 0 || o.recheck_cap < 0) return false;
    if (o.tests_per_lane < 0) return false;
    if (o.graph_levels < 0 || o.graph_levels > PC_MAX_LEVEL) return false;
    return true;
}

// Re-check queue capacity: the option, else sum of n^2 / 4 over the batch within [2^16, 2^25]
// (a level's tests grow with the pairs; borderline ones are a small fraction of them, largest
// with BF16x3, whose split error dominates its band).
int64_t rq_cap_of(const pc_options &o, double sum_n2) {
    if (o.recheck_cap > 0) return o.recheck_cap;
    return std::min<int64_t>((int64_t)1 << 25, std::max<int64_t>((int64_t)1 << 17, (int64_t)(sum_n2 / 4.0)));
}

int graph_levels_of(const pc_options &o) { return o.graph_levels > 0 ? o.graph_levels : 10; }

constexpr int kTailMaxLevel = 8;   // the tail kernel's deepest level (its register budget)

// Test budget of the tail kernel (0: not used). It is opt-in: one work-group per problem beats the
// level kernels only on the last few levels of a run, which the caller can tell from a first run.
long long tail_cap(const pc_options &o) {
    if (o.tail_tests <= 0 || o.force_recheck_all) return 0;
    return std::min<long long>(o.tail_tests, 1ll << 30);
}

// Standard normal CDF from erfc, and its inverse by Halley's method started from the rational
// approximation of Abramowitz & Stegun 26.2.23 (|error| < 4.5e-4); a few Halley steps reach full
// double precision. Only the lower tail is evaluated (p <= 0.5), so no cancellation occurs.
double phi_cdf(double x) { return 0.5 * std::erfc(-x / std::sqrt(2.0)); }

double phi_inv_lower(double p) {
    const double t = std::sqrt(-2.0 * std::log(p));
    double x = -(t - (2.515517 + 0.802853 * t + 0.010328 * t * t) /
                         (1.0 + 1.432788 * t + 0.189269 * t * t + 0.001308 * t * t * t));
    for (int it = 0; it < 4; ++it) {
        const double e = phi_cdf(x) - p;
        const double u = e * std::sqrt(2.0 * M_PI) * std::exp(0.5 * x * x);
        x = x - u / (1.0 + 0.5 * x * u);
    }
    return x;
}

// z = Phi^-1(1 - alpha/2) = -Phi^-1(alpha/2).
double z_of_alpha(double alpha) { return -phi_inv_lower(0.5 * alpha); }

double tau_of(double z, double m, int level) {
    const double dof = m - (double)level - 3.0;
    return dof > 0.0 ? z / std::sqrt(dof) : NAN;
}

// Bound on |C_low - C_fp64| for unit-norm columns (Cauchy-Schwarz bounds each sum of |products|
// by 1): FP32 rounding of Z (2u) plus sequential FP32 accumulation of mp terms (mp u); for the
// three BF16 products also the dropped lo*lo term and the split residuals (3 * 2^-18) over 3 mp
// accumulated terms.
// Bound on |C_low - C_64| for unit-norm standardized columns (every sum of |products| is <= 1 by
// Cauchy-Schwarz). The correlation kernel accumulates blocks of 16 (FP32) or 32 (BF16) samples
// from zero and adds the blocks with compensated summation, so:
//   FP32:   rounding Z to FP32 (2u per product), at most 2 roundings per product inside a block of
//           16 (32u), compensated summation of the blocks (2u), the stored FP32 value (u): 37u.
//   BF16x3: the dropped terms of z = hi + lo + r (|lo| <= 2^-8 |z|, |r| <= 2^-16 |z|):
//           lo*lo + hi*r + r*hi <= (3 + 2^-7) 2^-16; one block of 32 samples x 3 products with 2
//           roundings each (192u), compensated summation (2u), the stored value (u).
double eps_c_of(int prec, int64_t mp) {
    (void)mp;
    if (prec == PC_PREC_FP32) return 37.0 * kU32;
    if (prec == PC_PREC_BF16X3) return (3.0 + std::ldexp(1.0, -7)) * std::ldexp(1.0, -16) + 195.0 * kU32;
    return 0.0;
}

pc_status check_shape(int64_t n, int64_t m) {
    if (n < 2 || m < 4) return PC_ERR_SHAPE;
    if (n > (int64_t)1 << 16 || m > (int64_t)1 << 26) return PC_ERR_SHAPE;
    return PC_OK;
}

// ---------------------------------------------------------------------------------------------
// Workspace layout of a batch
// ---------------------------------------------------------------------------------------------
struct Region {
    size_t mu, inv, zt64, zlo, zhi, c, c64, adj, nbr, deg;
};

struct Plan {
    int count = 0;
    int prec = PC_PREC_FP32;
    size_t st = 0, table = 0, table_bytes = 0, nitems = 0, item_off = 0, rowdeg = 0, rq = 0, total = 0;
    int64_t rq_cap = 0;
    long long total_rows = 0, cs_blocks = 0, st_blocks = 0, tiles = 0;
    int64_t max_n = 0;
    std::vector<Region> reg;
    std::vector<long long> row_base, cs_base, st_base, tile_base;
};

// (n, m) of each problem; prec and rq_cap from the options.
Plan make_plan(const int64_t *ns, const int64_t *ms, int count, const pc_options &o) {
    Plan L;
    L.count = count;
    L.prec = o.precision;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off = align256(off + bytes); return at; };
    L.st = take(sizeof(DevState));
    L.table_bytes = sizeof(Prob) * count + 4 * sizeof(long long) * (count + 1);
    L.table = take(L.table_bytes);
    L.row_base.assign(count + 1, 0);
    L.cs_base.assign(count + 1, 0);
    L.st_base.assign(count + 1, 0);
    L.tile_base.assign(count + 1, 0);
    for (int d = 0; d < count; ++d) {
        const int64_t n = ns[d], mp = pad_m(ms[d]);
        L.row_base[d + 1] = L.row_base[d] + n;
        L.cs_base[d + 1] = L.cs_base[d] + cs_blocks(n);
        L.st_base[d + 1] = L.st_base[d] + st_blocks(n, mp);
        L.tile_base[d + 1] = L.tile_base[d] + corr_tiles(n);
        L.max_n = std::max(L.max_n, n);
    }
    L.total_rows = L.row_base[count];
    L.cs_blocks = L.cs_base[count];
    L.st_blocks = L.st_base[count];
    L.tiles = L.tile_base[count];
    double sum_n2 = 0.0;
    for (int d = 0; d < count; ++d) sum_n2 += (double)ns[d] * (double)ns[d];
    L.rq_cap = rq_cap_of(o, sum_n2);
    L.nitems = take(sizeof(long long) * (size_t)L.total_rows);
    L.item_off = take(sizeof(long long) * (size_t)(L.total_rows + 1));
    L.rowdeg = take(2 * sizeof(int) * (size_t)L.total_rows);
    L.rq = take(sizeof(RqEntry) * (size_t)L.rq_cap);
    L.reg.resize(count);
    for (int d = 0; d < count; ++d) {
        const size_t n = (size_t)ns[d], mp = (size_t)pad_m(ms[d]);
        Region &r = L.reg[d];
        r.mu = take(sizeof(double) * n);
        r.inv = take(sizeof(double) * n);
        r.zt64 = take(sizeof(double) * n * mp);
        r.zlo = take(L.prec == PC_PREC_FP32 ? sizeof(float) * n * mp
                     : L.prec == PC_PREC_BF16X3 ? sizeof(uint16_t) * n * mp : 0);
        r.zhi = take(L.prec == PC_PREC_BF16X3 ? sizeof(uint16_t) * n * mp : 0);
        r.c = take((L.prec == PC_PREC_FP64 ? sizeof(double) : sizeof(float)) * n * n);
        // FP64 copy of C for a level whose FP32 re-check queue overflows (redone in FP64)
        r.c64 = take(L.prec == PC_PREC_FP64 ? 0 : sizeof(double) * n * n);
        r.adj = take(sizeof(unsigned long long) * n * (size_t)words_per_row((int64_t)n));
        r.nbr = take(sizeof(int32_t) * n * n);
        r.deg = take(sizeof(int32_t) * n);
    }
    L.total = off;
    return L;
}

// Host image of the problem table for the given workspace base.
// m_nominal > 0 replaces the sample size in the thresholds tau_l (a correlation matrix given by the
// caller: there is no data, and m may be a nominal large-sample value).
void fill_probs(const pc_ctx *ctx, const Plan &L, unsigned char *ws, const pc_problem *pp,
                std::vector<Prob> &out, double m_nominal = -1.0) {
    out.assign(L.count, Prob{});
    for (int d = 0; d < L.count; ++d) {
        Prob &P = out[d];
        const Region &r = L.reg[d];
        std::memset(&P, 0, sizeof(P));
        P.n = pp[d].n;
        P.m = pp[d].m;
        P.mp = pad_m(P.m);
        P.W = words_per_row(P.n);
        P.X = pp[d].X;
        P.mu = reinterpret_cast<double *>(ws + r.mu);
        P.inv = reinterpret_cast<double *>(ws + r.inv);
        P.zt64 = reinterpret_cast<double *>(ws + r.zt64);
        P.zlo = ws + r.zlo;
        P.zhi = ws + r.zhi;
        P.C = ws + r.c;
        P.adj = pp[d].adj_out ? reinterpret_cast<unsigned long long *>(pp[d].adj_out)
                              : reinterpret_cast<unsigned long long *>(ws + r.adj);
        P.nbr = reinterpret_cast<int *>(ws + r.nbr);
        P.deg = reinterpret_cast<int *>(ws + r.deg);
        P.recs = pp[d].sep.recs;
        P.rec_cap = pp[d].sep.cap;
        P.rec_count = reinterpret_cast<long long *>(pp[d].sep.count);
        P.max_level = pp[d].max_level >= 0 ? std::min(pp[d].max_level, PC_MAX_LEVEL + 1) : PC_MAX_LEVEL + 1;
        const double z = z_of_alpha(pp[d].alpha);
        const double m_tau = m_nominal > 0.0 ? m_nominal : (double)P.m;
        for (int l = 0; l < kLevels; ++l) {
            P.tau[l] = tau_of(z, m_tau, l);
            P.t[l] = std::isnan(P.tau[l]) ? 0.0f : (float)std::tanh(P.tau[l]);
            const double eps = eps_c_of(L.prec, P.mp) + (4.0 * l + 16.0) * kU32;
            P.band[l] = (float)((double)ctx->opt.margin_scale * eps);
        }
        P.t0 = std::tanh(P.tau[0]);
        P.eps_c = eps_c_of(L.prec, P.mp);
    }
}

Batch make_batch(const pc_ctx *ctx, const Plan &L, unsigned char *ws) {
    Batch b{};
    b.rank_lo = 0;
    b.rank_hi = ~0ull;
    b.probe = 0;
    b.l1_perm = 0;
    b.corr_only = 0;
    b.probs = reinterpret_cast<Prob *>(ws + L.table);
    b.count = L.count;
    b.prec = L.prec;
    b.force_recheck = L.prec != PC_PREC_FP64 && ctx->opt.force_recheck_all;
    const long long groups = ctx->level_grid[1] > 0 ? ctx->level_grid[1] : 4 * ctx->num_cu;
    b.lane_tests = ctx->opt.tests_per_lane > 0 ? ctx->opt.tests_per_lane
                                               : (L.total_rows <= groups ? kAutoLaneTestsSmall : kAutoLaneTests);
    b.set_lanes = 4;
    const long long *bases = reinterpret_cast<const long long *>(ws + L.table + sizeof(Prob) * L.count);
    b.row_base = bases;
    b.cs_base = bases + (L.count + 1);
    b.st_base = bases + 2 * (L.count + 1);
    b.tile_base = bases + 3 * (L.count + 1);
    b.nitems = reinterpret_cast<long long *>(ws + L.nitems);
    b.item_off = reinterpret_cast<long long *>(ws + L.item_off);
    b.rowdeg = reinterpret_cast<int *>(ws + L.rowdeg);
    b.binom = ctx->binom;
    b.st = reinterpret_cast<DevState *>(ws + L.st);
    b.rq = reinterpret_cast<RqEntry *>(ws + L.rq);
    b.rq_cap = L.rq_cap;
    b.total_rows = L.total_rows;
    return b;
}

pc_status ensure_binom(pc_ctx *ctx, int64_t max_n) {
    if (max_n + 1 <= ctx->binom_rows) return PC_OK;
    const int64_t rows = std::max<int64_t>(max_n + 1, 2 * ctx->binom_rows);
    unsigned long long *t = nullptr;
    PC_HIP(hipStreamSynchronize(ctx->stream));
    PC_HIP(hipMalloc(&t, sizeof(unsigned long long) * rows * kBinomCols));
    if (ctx->binom) (void)hipFree(ctx->binom);
    ctx->binom = t;
    ctx->binom_rows = rows;
    PC_HIP(launch_binom(ctx->stream, t, rows));
    return PC_OK;
}

// Copies the problem table into the workspace (stream ordered, from pinned staging).
pc_status upload_table(pc_ctx *ctx, const Plan &L, unsigned char *ws, const std::vector<Prob> &probs) {
    if (ctx->staging_pending) {
        PC_HIP(hipEventSynchronize(ctx->staging_done));
        ctx->staging_pending = false;
    }
    if (L.table_bytes > ctx->staging_bytes) {
        if (ctx->staging) (void)hipHostFree(ctx->staging);
        ctx->staging = nullptr;
        ctx->staging_bytes = 0;
        const size_t want = std::max(L.table_bytes, (size_t)1 << 16);
        PC_HIP(hipHostMalloc(&ctx->staging, want, hipHostMallocDefault));
        ctx->staging_bytes = want;
    }
    unsigned char *h = static_cast<unsigned char *>(ctx->staging);
    std::memcpy(h, probs.data(), sizeof(Prob) * L.count);
    long long *bases = reinterpret_cast<long long *>(h + sizeof(Prob) * L.count);
    const size_t nb = (size_t)L.count + 1;
    std::memcpy(bases, L.row_base.data(), sizeof(long long) * nb);
    std::memcpy(bases + nb, L.cs_base.data(), sizeof(long long) * nb);
    std::memcpy(bases + 2 * nb, L.st_base.data(), sizeof(long long) * nb);
    std::memcpy(bases + 3 * nb, L.tile_base.data(), sizeof(long long) * nb);
    PC_HIP(hipMemcpyAsync(ws + L.table, h, L.table_bytes, hipMemcpyHostToDevice, ctx->stream));
    PC_HIP(hipEventRecord(ctx->staging_done, ctx->stream));
    ctx->staging_pending = true;
    return PC_OK;
}

// A tuned per-level value, or 0 (lds_budget: -1) when the level keeps the context's.
int tuned_at(const pc_ctx *ctx, const int32_t (&v)[PC_MAX_LEVEL + 1], int level, int none) {
    return ctx->tuned && level >= 1 && level <= PC_MAX_LEVEL ? v[level] : none;
}

// Conditioning-set ranks per work item. Levels up to kFastLevels give every thread its own sets;
// deeper levels give every wavefront one set at a time, so their items are much smaller.
int ranks_per_item(const pc_ctx *ctx, int level) {
    const int t = tuned_at(ctx, ctx->tuning.ranks_per_lane, level, 0);
    const int o = t > 0 ? t : ctx->opt.ranks_per_lane;
    if (level > kFastLevels) return 4 * (o > 0 ? o : 4);
    // Sets per lane: one at level 1 (a set there is a single division), several while a set's
    // factor is cheap, one again once it is long (l^3 work per set at deep levels).
    const int q = o > 0 ? o : (level == 1 ? 1 : (level <= 3 ? 4 : (level <= 7 ? 2 : 1)));
    return q * kLevelThreads;
}

// The batch of one level's launches: its item size bound (planning and level kernels must agree).
Batch at_level(const pc_ctx *ctx, Batch b, int level) {
    const int t = tuned_at(ctx, ctx->tuning.tests_per_lane, level, 0);
    if (t > 0) b.lane_tests = t;
    const int sl = tuned_at(ctx, ctx->tuning.set_lanes, level, 0);
    b.set_lanes = sl > 0 ? sl : 4;
    return b;
}

// Dynamic LDS of a level launch: the kernel's fixed part for its precision (the context's, or
// FP64 for a promoted level) and the row-staging budget (the level's tuned one, if any).
int level_lds_bytes(const pc_ctx *ctx, int prec = -1, int level = 0) {
    const size_t fixed = level_lds_fixed(prec >= 0 ? prec : ctx->opt.precision);
    const int tb = tuned_at(ctx, ctx->tuning.lds_budget, level, -1);
    size_t budget = (size_t)(tb >= 0 ? tb : ctx->opt.lds_budget);
    const size_t limit = 60 * 1024 - fixed;  // with the kernel's static staging, within 64 KiB
    if (budget > limit) budget = limit;
    return (int)(fixed + budget);
}

// Work-groups of a level launch: the option, else all that fit at once with the launch's LDS.
int auto_grid(const pc_ctx *ctx, int level, int prec = -1) {
    if (ctx->opt.grid > 0) return ctx->opt.grid;
    const int tg = tuned_at(ctx, ctx->tuning.grid, level, 0);
    if (tg > 0) return tg;
    const int p = prec >= 0 ? prec : ctx->opt.precision;
    int g = ctx->level_grid[level];
    if (p != ctx->opt.precision || tuned_at(ctx, ctx->tuning.lds_budget, level, -1) >= 0) {
        const int nb = level_blocks_per_cu(p, level, level_lds_bytes(ctx, p, level));
        g = nb > 0 ? nb * ctx->num_cu : 0;
    }
    return g > 0 ? g : 2 * ctx->num_cu;
}

// Work-groups of a level's re-check launch: the tuned number, else 4 per CU.
int recheck_grid_at(const pc_ctx *ctx, int level) {
    const int t = tuned_at(ctx, ctx->tuning.recheck_grid, level, 0);
    return t > 0 ? t : ctx->recheck_grid;
}

void reset_timed(pc_ctx *ctx) {
    ctx->rec_compact = ctx->rec_level = ctx->rec_recheck = 0ull;
    ctx->rec_prep = ctx->rec_corr = false;
}

// Milliseconds between two events recorded by the current call (0 if the query fails; its error is
// cleared, so that the next launch's hipGetLastError does not report it).
float event_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();
        ms = 0.f;
    }
    return ms;
}

bool timed(const pc_ctx *ctx, int bit, bool capturing) { return !capturing && (ctx->opt.timing & bit); }

// Level kernels of level l are timed: every level (bit 2) or level 1 alone (bit 32). Not inside a
// captured graph (an event recorded during capture only marks a dependency, it is not re-recorded
// by the replays).
bool timed_level(const pc_ctx *ctx, int level, bool capturing) {
    return timed(ctx, 2, capturing) || (level == 1 && timed(ctx, 32, capturing));
}

// Standardize + correlation + level 0 for every problem of the batch.
pc_status enqueue_corr(pc_ctx *ctx, const Batch &b, const Plan &L, bool capturing) {
    hipStream_t s = ctx->stream;
    PC_HIP(launch_init(s, b));
    if (timed(ctx, 16, capturing)) PC_HIP(hipEventRecord(ctx->ev_prep[0], s));
    PC_HIP(launch_colstats(s, b, L.cs_blocks));
    PC_HIP(launch_standardize(s, b, L.st_blocks));
    if (timed(ctx, 16, capturing)) {
        PC_HIP(hipEventRecord(ctx->ev_prep[1], s));
        ctx->rec_prep = true;
    }
    if (timed(ctx, 1, capturing)) PC_HIP(hipEventRecord(ctx->ev_corr[0], s));
    PC_HIP(launch_corr(s, b, L.tiles, ctx->num_cu));
    if (timed(ctx, 1, capturing)) {
        PC_HIP(hipEventRecord(ctx->ev_corr[1], s));
        ctx->rec_corr = true;
    }
    return PC_OK;
}

struct OrderRun {
    const pc_order *order;
    const Plan *L;
    unsigned char *ws;
};

constexpr int kProbeMaxLevel = 8;

// Whether the shared-set order runs at level 1: a row model, or the |C_ik| ranking.
bool row_order_on(const pc_order *o) { return o->row_params || (o->row_rank == 1 && o->row_top > 0); }

// Whether level l runs the probe pass of the ordering.
bool probe_level(const pc_order *o, int level) {
    if (!o->params) return false;
    const int hi = o->max_level > 0 ? o->max_level : kProbeMaxLevel;
    return level >= o->min_level && level <= hi && level <= kProbeMaxLevel && level <= o->top;
}

// Whether the tail kernel may take over from `level`: enabled, and no per-edge probe pass would
// have run at that level or later.
bool tail_allowed(const pc_ctx *ctx, const OrderRun *ord, int level) {
    if (tail_cap(ctx->opt) <= 0 || level < 2 || level > kTailMaxLevel) return false;
    return !(ord && ord->order->params);
}

// Compaction and planning of one level: the snapshot G' and the work plan (and the stop rule's
// maximum degree) of every problem. Level PC_MAX_LEVEL + 1 is planned only, to tell whether the
// level cap stopped a run.
pc_status enqueue_plan(pc_ctx *ctx, const Batch &b_in, int level, bool capturing) {
    hipStream_t s = ctx->stream;
    const Batch b = at_level(ctx, b_in, level);
    const int R = ranks_per_item(ctx, level <= PC_MAX_LEVEL ? level : PC_MAX_LEVEL);
    if (timed(ctx, 4, capturing)) PC_HIP(hipEventRecord(ctx->ev_compact[level][0], s));
    PC_HIP(launch_compact(s, b, level, R));
    PC_HIP(launch_plan(s, b, level));
    if (timed(ctx, 4, capturing)) {
        PC_HIP(hipEventRecord(ctx->ev_compact[level][1], s));
        ctx->rec_compact |= 1ull << level;
    }
    return PC_OK;
}

// (Probe pass,) CI tests and FP64 re-check of a planned level.
pc_status enqueue_run(pc_ctx *ctx, const Batch &b_in, int level, bool capturing, const OrderRun *ord) {
    hipStream_t s = ctx->stream;
    const Batch b = at_level(ctx, b_in, level);
    const int R = ranks_per_item(ctx, level);
    // Probe pass of the learned ordering: the best-scored subsets of every edge, before the plain
    // enumeration of the same level.
    const bool row_order = ord && level == 1 && row_order_on(ord->order);
    if (ord && probe_level(ord->order, level) && !row_order)
        PC_HIP(launch_probe(s, b, level, ord->order->params, ord->order->top, ctx->num_cu));
    if (timed_level(ctx, level, capturing)) PC_HIP(hipEventRecord(ctx->ev_level[level][0], s));
    if (row_order) {
        // Shared-set order: each row's best-scored candidates move to the front of its neighbour
        // list and their sets are tested first (in the ordering kernel), then the level kernel runs
        // the remaining ranks; together they cover every set of the level once, on the same G'.
        const int T = ord->order->row_top;
        PC_HIP(launch_row_order(s, b, level, ord->order->row_params, T, ord->order->row_rank,
                                ord->order->row_short, ord->order->row_sort, ctx->num_cu));
        // The remaining ranks in one pass, or two (the strongest sets of every row first).
        const int split = ord->order->row_split;
        Batch bm = b;
        bm.l1_perm = ord->order->row_sort;
        bm.rank_lo = (unsigned long long)T;
        if (split > T) {
            bm.rank_hi = (unsigned long long)split;
            PC_HIP(launch_window(s, bm, level, R));
            PC_HIP(launch_level(s, bm, level, R, level_lds_bytes(ctx, b.prec, level), auto_grid(ctx, level, b.prec)));
            bm.rank_lo = (unsigned long long)split;
            bm.rank_hi = ~0ull;
        }
        PC_HIP(launch_window(s, bm, level, R));
        PC_HIP(launch_level(s, bm, level, R, level_lds_bytes(ctx, b.prec, level), auto_grid(ctx, level, b.prec)));
    } else {
        PC_HIP(launch_level(s, b, level, R, level_lds_bytes(ctx, b.prec, level), auto_grid(ctx, level, b.prec)));
    }
    if (timed_level(ctx, level, capturing)) {
        PC_HIP(hipEventRecord(ctx->ev_level[level][1], s));
        ctx->rec_level |= 1ull << level;
    }
    if (timed(ctx, 8, capturing)) PC_HIP(hipEventRecord(ctx->ev_recheck[level][0], s));
    PC_HIP(launch_recheck(s, b, level, recheck_grid_at(ctx, level)));
    if (timed(ctx, 8, capturing)) {
        PC_HIP(hipEventRecord(ctx->ev_recheck[level][1], s));
        ctx->rec_recheck |= 1ull << level;
    }
    ctx->top_run = std::max(ctx->top_run, level);
    return PC_OK;
}

// Compaction, planning, (probe pass,) CI tests and FP64 re-check of one level.
pc_status enqueue_level(pc_ctx *ctx, const Batch &b, int level, bool capturing, const OrderRun *ord = nullptr) {
    pc_status st = enqueue_plan(ctx, b, level, capturing);
    if (st != PC_OK || level > PC_MAX_LEVEL) return st;
    return enqueue_run(ctx, b, level, capturing, ord);
}

// Copies the problem table and queue state back (synchronising the stream).
pc_status read_table(pc_ctx *ctx, const Plan &L, unsigned char *ws, std::vector<Prob> &host, DevState &ds) {
    host.resize(L.count);
    PC_HIP(hipMemcpyAsync(host.data(), ws + L.table, sizeof(Prob) * L.count, hipMemcpyDeviceToHost, ctx->stream));
    PC_HIP(hipMemcpyAsync(&ds, ws + L.st, sizeof(DevState), hipMemcpyDeviceToHost, ctx->stream));
    PC_HIP(hipStreamSynchronize(ctx->stream));
    return PC_OK;
}

// Levels from..top on the stream, level `from` already planned. The stop rule runs on the device;
// the host only bounds how far to enqueue: degrees never grow, so a problem whose G' at level l has
// maximum degree D needs no level past D - 1. The bound is read after planning `from` and, on long
// runs, again every few levels.
pc_status run_levels_eager(pc_ctx *ctx, const Batch &b, const Plan &L, unsigned char *ws, int from, int top,
                           const OrderRun *ord) {
    std::vector<Prob> host;
    DevState ds;
    int l = from;
    int tail_after = 1;   // the tail kernel is tried only above the level where it last stopped
    while (l <= top) {
        pc_status s = read_table(ctx, L, ws, host, ds);
        if (s != PC_OK) return s;
        if (ds.done) break;
        int last = 0;
        long long est = 0;   // bound on the tests of level l: items x sets per item x candidates
        for (const Prob &P : host) {
            const int md = P.maxdeg[l];
            if (md - 1 >= l) last = std::max(last, std::min(std::min(P.max_level, PC_MAX_LEVEL + 1), md - 1));
            if (l <= PC_MAX_LEVEL) est += P.items[l] * (long long)ranks_per_item(ctx, l) * std::max(md - l, 0);
        }
        if (last < l) break;
        if (l > tail_after && l <= top && tail_allowed(ctx, ord, l) && est <= tail_cap(ctx->opt)) {
            // Few tests left: the rest of every problem in one work-group each; problems the tail
            // leaves at a larger level continue here from the smallest such level.
            PC_HIP(launch_tail(ctx->stream, b, l, tail_cap(ctx->opt)));
            if ((s = read_table(ctx, L, ws, host, ds)) != PC_OK) return s;
            int next = 0;
            for (const Prob &P : host)
                if (P.tail_next > 0) next = next == 0 ? P.tail_next : std::min(next, P.tail_next);
            if (next == 0 || next > top) break;
            tail_after = next;
            l = next;
            if ((s = enqueue_plan(ctx, b, l, false)) != PC_OK) return s;
            continue;
        }
        const int upto = std::min(top, last - l >= 6 ? l + 3 : last);
        for (; l <= upto; ++l) {
            if (l <= PC_MAX_LEVEL && (s = enqueue_run(ctx, b, l, false, ord)) != PC_OK) return s;
            if (l + 1 <= top && (s = enqueue_plan(ctx, b, l + 1, false)) != PC_OK) return s;
        }
    }
    return PC_OK;
}

// Levels (after level 0) to enqueue: up to the largest cap of the batch; a cap above PC_MAX_LEVEL
// adds one planning-only pass that tells whether the level cap stopped a problem.
int levels_to_enqueue(const pc_problem *pp, int count) {
    int top = 0;
    for (int d = 0; d < count; ++d) {
        const int cap = pp[d].max_level >= 0 ? std::min(pp[d].max_level, PC_MAX_LEVEL + 1) : PC_MAX_LEVEL + 1;
        top = std::max(top, cap);
    }
    return top;
}

// Per-problem result from the device statistics (after the stream has completed). A problem ran
// level l iff G' of l had a node with at least l + 1 neighbours and l was enabled (within its cap,
// PC_MAX_LEVEL, and m - l - 3 > 0); the first level that did not run tells why it stopped.
pc_status problem_result(const Prob &P, const DevState &ds, pc_run_stats *st) {
    int levels_run = 1;
    pc_status res = PC_OK;
    for (int l = 1; l <= PC_MAX_LEVEL + 1; ++l) {
        const bool enough = P.maxdeg[l] >= l + 1;
        const bool enabled = l <= P.max_level && l <= PC_MAX_LEVEL && !std::isnan(P.tau[l]);
        if (enough && enabled) {
            levels_run = l + 1;
            continue;
        }
        if (enough && l <= P.max_level) {
            if (l > PC_MAX_LEVEL) res = PC_WARN_LEVEL_CAP;
            else if (std::isnan(P.tau[l])) res = PC_WARN_SAMPLE_LIMIT;
        }
        break;
    }
    if (st) {
        std::memset(st, 0, sizeof(*st));
        for (int l = 0; l <= PC_MAX_LEVEL; ++l) {
            st->tests[l] = P.tests[l];
            st->removed[l] = P.removed[l];
            st->rechecks[l] = P.rechecks[l];
            st->items[l] = P.items[l];
            st->audit_violations[l] = P.audit_viol[l];
            st->probe_tests[l] = P.probe_tests[l];
            st->probe_removed[l] = P.probe_removed[l];
            st->max_degree[l] = l == 0 ? 0 : P.maxdeg[l];
        }
        st->levels_run = levels_run;
    }
    if (P.err) return (pc_status)P.err;
    if (ds.overflow) return PC_ERR_UNSUPPORTED;
    if (ds.rq_overflow || ds.rq_overflow_tail) return PC_ERR_WORKSPACE;
    return res;
}

// Results of every problem from a downloaded table (SepSet counts are read per problem).
pc_status results(const std::vector<Prob> &host, const DevState &ds, pc_run_stats *st, pc_status *status) {
    pc_status first = PC_OK;
    for (size_t d = 0; d < host.size(); ++d) {
        pc_status r = problem_result(host[d], ds, st ? &st[d] : nullptr);
        if (r >= 0 && host[d].rec_count) {
            long long cnt = 0;
            PC_HIP(hipMemcpy(&cnt, host[d].rec_count, sizeof(cnt), hipMemcpyDeviceToHost));
            if (cnt > host[d].rec_cap) r = PC_ERR_SEPSET_CAPACITY;
        }
        if (status) status[d] = r;
        if (r < 0 && first >= 0) first = r;
        if (r > 0 && first == PC_OK) first = r;
    }
    return first;
}

// Copies the problem table and queue state back (synchronising) and fills per-problem results.
pc_status collect(pc_ctx *ctx, size_t table_off, size_t st_off, int count, unsigned char *ws,
                  pc_run_stats *st, pc_status *status, std::vector<Prob> &host, DevState *ds_out = nullptr) {
    host.resize(count);
    DevState ds;
    PC_HIP(hipMemcpyAsync(host.data(), ws + table_off, sizeof(Prob) * count, hipMemcpyDeviceToHost, ctx->stream));
    PC_HIP(hipMemcpyAsync(&ds, ws + st_off, sizeof(DevState), hipMemcpyDeviceToHost, ctx->stream));
    PC_HIP(hipStreamSynchronize(ctx->stream));
    if (ds_out) *ds_out = ds;
    return results(host, ds, st, status);
}

void fill_times(pc_ctx *ctx, pc_run_stats *st, int top_level) {
    if (!st || !ctx->opt.timing) return;
    const int tm = ctx->opt.timing;
    if ((tm & 16) && ctx->rec_prep) st->prep_ms = event_ms(ctx->ev_prep[0], ctx->ev_prep[1]);
    if ((tm & 1) && ctx->rec_corr) st->corr_ms = event_ms(ctx->ev_corr[0], ctx->ev_corr[1]);
    for (int l = 1; l <= std::min(top_level, PC_MAX_LEVEL); ++l) {
        const unsigned long long bit = 1ull << l;
        if ((tm & 4) && (ctx->rec_compact & bit)) st->compact_ms[l] = event_ms(ctx->ev_compact[l][0], ctx->ev_compact[l][1]);
        if (((tm & 2) || ((tm & 32) && l == 1)) && (ctx->rec_level & bit))
            st->level_ms[l] = event_ms(ctx->ev_level[l][0], ctx->ev_level[l][1]);
        if ((tm & 8) && (ctx->rec_recheck & bit)) st->recheck_ms[l] = event_ms(ctx->ev_recheck[l][0], ctx->ev_recheck[l][1]);
    }
}

pc_status check_ws(void *ws, size_t ws_bytes, const Plan &L) {
    if (!ws) return PC_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return PC_ERR_INVALID_ARG;
    if (ws_bytes < L.total) return PC_ERR_WORKSPACE;
    return PC_OK;
}

pc_status check_problem(const pc_problem &p) {
    if (!p.X || !p.adj_out || !p.sep.count || (!p.sep.recs && p.sep.cap > 0)) return PC_ERR_INVALID_ARG;
    if (!(p.alpha > 0.0 && p.alpha < 1.0)) return PC_ERR_INVALID_ARG;
    return check_shape(p.n, p.m);
}

Plan plan_of(const pc_problem *pp, int count, const pc_options &o) {
    std::vector<int64_t> ns(count), ms(count);
    for (int d = 0; d < count; ++d) { ns[d] = pp[d].n; ms[d] = pp[d].m; }
    return make_plan(ns.data(), ms.data(), count, o);
}

// Every launch of the batched skeletons (the table must already be uploaded).
pc_status enqueue_skeletons(pc_ctx *ctx, const pc_problem *pp, int count, const Plan &L,
                            unsigned char *ws, bool capturing, const pc_order *order = nullptr,
                            bool given_c = false) {
    const Batch b = make_batch(ctx, L, ws);
    pc_status s = PC_OK;
    reset_timed(ctx);
    if (given_c) {
        // C is already in the workspace: level 0 reads it directly.
        PC_HIP(launch_init(ctx->stream, b));
        if (timed(ctx, 1, capturing)) PC_HIP(hipEventRecord(ctx->ev_corr[0], ctx->stream));
        PC_HIP(launch_level0_given(ctx->stream, b));
        if (timed(ctx, 1, capturing)) {
            PC_HIP(hipEventRecord(ctx->ev_corr[1], ctx->stream));
            ctx->rec_corr = true;
        }
    } else if ((s = enqueue_corr(ctx, b, L, capturing)) != PC_OK) {
        return s;
    }
    const OrderRun ord{order, &L, ws};
    const OrderRun *po = order ? &ord : nullptr;
    const int top = levels_to_enqueue(pp, count);
    ctx->top_run = 0;
    ctx->tail_enqueued = false;
    if (capturing) {
        // A graph holds levels 1..G and then either the tail kernel from G + 1 (which runs the
        // rest while levels stay small) or the planning of G + 1; pc_graph_results continues
        // whatever is left.
        const int G = std::min(top, graph_levels_of(ctx->opt));
        for (int l = 1; l <= G; ++l)
            if ((s = enqueue_level(ctx, b, l, true, po)) != PC_OK) return s;
        if (G < top) {
            if (tail_allowed(ctx, po, G + 1)) {
                PC_HIP(launch_tail(ctx->stream, b, G + 1, tail_cap(ctx->opt)));
                ctx->tail_enqueued = true;
            } else if ((s = enqueue_plan(ctx, b, G + 1, true)) != PC_OK) {
                return s;
            }
        }
        return PC_OK;
    }
    if (top < 1) return PC_OK;
    if ((s = enqueue_level(ctx, b, 1, false, po)) != PC_OK) return s;
    if (top < 2) return PC_OK;
    if ((s = enqueue_plan(ctx, b, 2, false)) != PC_OK) return s;
    return run_levels_eager(ctx, b, L, ws, 2, top, po);
}

// The FP32 (or BF16x3) re-check queue of `level` overflowed, so the device stopped the level loop
// after that level with some borderline tests undecided. Every decision that was made is exact
// (outside the error band, or re-checked in FP64), so the level is completed by testing it again in
// FP64: C in FP64 from the standardized data (the GEMM without its level-0 epilogue), the level's
// sets over its own snapshot G' (still in the neighbour lists: no later compaction ran), and the
// remaining levels in FP64 as well. Removals already made, and their SepSets, stand.
pc_status promote_fp64(pc_ctx *ctx, const Plan &L, unsigned char *ws, std::vector<Prob> &host, int level, int top) {
    hipStream_t s = ctx->stream;
    for (int d = 0; d < L.count; ++d) host[d].C = ws + L.reg[d].c64;
    pc_status st = upload_table(ctx, L, ws, host);
    if (st != PC_OK) return st;
    Batch b = make_batch(ctx, L, ws);
    b.prec = PC_PREC_FP64;
    Batch bc = b;
    bc.corr_only = 1;
    PC_HIP(launch_corr(s, bc, L.tiles, ctx->num_cu));
    PC_HIP(launch_rearm(s, b));
    const int R = ranks_per_item(ctx, level);
    const Batch bl = at_level(ctx, b, level);
    PC_HIP(launch_window(s, bl, level, R));
    PC_HIP(launch_level(s, bl, level, R, level_lds_bytes(ctx, PC_PREC_FP64, level), auto_grid(ctx, level, PC_PREC_FP64)));
    PC_HIP(launch_recheck(s, b, level, recheck_grid_at(ctx, level)));
    ctx->top_run = std::max(ctx->top_run, level);
    if (level >= top) return PC_OK;
    if ((st = enqueue_plan(ctx, b, level + 1, false)) != PC_OK) return st;
    return run_levels_eager(ctx, b, L, ws, level + 1, top, nullptr);
}

// collect(), after completing in FP64 a level whose re-check queue overflowed (see promote_fp64).
// *promoted: 0, or the level from which the run went on in FP64 (also in every st[d].fp64_from).
pc_status collect_promoting(pc_ctx *ctx, const Plan &L, unsigned char *ws, int top, pc_run_stats *st,
                            pc_status *status, std::vector<Prob> &host, int *promoted = nullptr) {
    DevState ds;
    if (promoted) *promoted = 0;
    const pc_status r = collect(ctx, L.table, L.st, L.count, ws, st, status, host, &ds);
    if (L.prec == PC_PREC_FP64 || ds.rq_overflow <= 0 || ds.rq_overflow_tail || r == PC_ERR_HIP) return r;
    const pc_status s = promote_fp64(ctx, L, ws, host, ds.rq_overflow, top);
    if (s != PC_OK) return s;
    pc_status s2;
    const pc_status r2 = collect(ctx, L.table, L.st, L.count, ws, st, status, host);
    // The table points at the plan's own C again (a captured graph replays with it).
    for (int d = 0; d < L.count; ++d) host[d].C = ws + L.reg[d].c;
    if (r2 != PC_ERR_HIP && (s2 = upload_table(ctx, L, ws, host)) != PC_OK) return s2;
    if (st)
        for (int d = 0; d < L.count; ++d) st[d].fp64_from = ds.rq_overflow;
    if (promoted) *promoted = ds.rq_overflow;
    return r2;
}

bool valid_order(const pc_order *o) {
    if (!o || (!o->params && !row_order_on(o))) return false;
    if (o->params && !(o->min_level >= 1 && o->min_level <= kProbeMaxLevel && o->top >= 1 && o->top <= 8 &&
                       (o->max_level == 0 || (o->max_level >= o->min_level && o->max_level <= kProbeMaxLevel))))
        return false;
    if (o->row_rank != 0 && o->row_rank != 1) return false;
    if (row_order_on(o)) {
        if (!(o->row_top >= 1 && o->row_top <= 16)) return false;
        if ((o->row_sort != 0 && o->row_sort != 1) || o->row_split < 0) return false;
        if (o->row_short != 0 && (o->row_rank != 0 || o->row_short < o->row_top || o->row_short > 64)) return false;
    }
    return true;
}

// Validates a batch and prepares its table in the workspace.
pc_status prepare(pc_ctx *ctx, const pc_problem *probs, int count, void *ws, size_t ws_bytes,
                  Plan &L, std::vector<Prob> &table) {
    pc_status s;
    int64_t max_n = 0;
    for (int d = 0; d < count; ++d) {
        if ((s = check_problem(probs[d])) != PC_OK) return s;
        max_n = std::max(max_n, probs[d].n);
    }
    L = plan_of(probs, count, ctx->opt);
    if ((s = check_ws(ws, ws_bytes, L)) != PC_OK) return s;
    if ((s = ensure_binom(ctx, max_n)) != PC_OK) return s;
    fill_probs(ctx, L, static_cast<unsigned char *>(ws), probs, table);
    return upload_table(ctx, L, static_cast<unsigned char *>(ws), table);
}

}  // namespace

extern "C" {

pc_status pc_default_options(pc_options *opt) {
    if (!opt) return PC_ERR_INVALID_ARG;
    *opt = defaults();
    return PC_OK;
}

void pc_destroy(pc_ctx *ctx) {
    if (!ctx) return;
    auto rm = [](hipEvent_t e) { if (e) (void)hipEventDestroy(e); };
    for (auto e : ctx->ev_prep) rm(e);
    for (auto e : ctx->ev_corr) rm(e);
    for (int l = 0; l < kLevels; ++l)
        for (int k = 0; k < 2; ++k) { rm(ctx->ev_compact[l][k]); rm(ctx->ev_level[l][k]); rm(ctx->ev_recheck[l][k]); }
    rm(ctx->staging_done);
    if (ctx->binom) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(ctx->binom);
    }
    if (ctx->staging) (void)hipHostFree(ctx->staging);
    delete ctx;
}

pc_status pc_create(pc_ctx **out, void *stream, const pc_options *opt) {
    if (!out) return PC_ERR_INVALID_ARG;
    *out = nullptr;
    pc_options o = opt ? *opt : defaults();
    if (!valid_options(o)) return PC_ERR_INVALID_ARG;
    int dev = 0;
    PC_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    PC_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return PC_ERR_UNSUPPORTED;
    pc_ctx *c = new (std::nothrow) pc_ctx();
    if (!c) return PC_ERR_HIP;
    c->stream = static_cast<hipStream_t>(stream);
    c->opt = o;
    c->device = dev;
    c->num_cu = prop.multiProcessorCount;
    bool ok = true;
    auto mk = [&](hipEvent_t &e) { if (hipEventCreate(&e) != hipSuccess) { e = nullptr; ok = false; } };
    for (auto &e : c->ev_prep) mk(e);
    for (auto &e : c->ev_corr) mk(e);
    for (int l = 0; l < kLevels; ++l)
        for (int k = 0; k < 2; ++k) { mk(c->ev_compact[l][k]); mk(c->ev_level[l][k]); mk(c->ev_recheck[l][k]); }
    if (hipEventCreateWithFlags(&c->staging_done, hipEventDisableTiming) != hipSuccess) {
        c->staging_done = nullptr;
        ok = false;
    }
    // Level kernels launch as many work-groups as fit on the device at once (persistent workers).
    for (int l = 0; l < kLevels; ++l) {
        const int nb = l >= 1 && l <= PC_MAX_LEVEL ? level_blocks_per_cu(o.precision, l, level_lds_bytes(c)) : 0;
        c->level_grid[l] = nb > 0 ? nb * c->num_cu : 0;
    }
    {
        const int nb = recheck_blocks_per_cu();
        c->recheck_grid = (nb > 0 ? std::min(nb, 4) : 4) * c->num_cu;
    }
    if (ok && ensure_binom(c, 8191) != PC_OK) ok = false;
    if (ok && scratch_address(dev, &c->scratch) != PC_OK) ok = false;
    // Pinned staging for problem tables, so that single-problem calls need no allocation later.
    if (ok) {
        if (hipHostMalloc(&c->staging, (size_t)1 << 16, hipHostMallocDefault) == hipSuccess) c->staging_bytes = (size_t)1 << 16;
        else ok = false;
    }
    if (ok && hipStreamSynchronize(c->stream) != hipSuccess) ok = false;
    if (!ok) {
        pc_destroy(c);
        return PC_ERR_HIP;
    }
    *out = c;
    return PC_OK;
}

size_t pc_workspace_bytes(int64_t n, int64_t m, const pc_options *opt) {
    pc_options o = opt ? *opt : defaults();
    if (n < 1 || m < 1) return 0;
    return make_plan(&n, &m, 1, o).total;
}

size_t pc_batch_workspace_bytes(const pc_problem *probs, int count, const pc_options *opt) {
    pc_options o = opt ? *opt : defaults();
    if (!probs || count < 1) return 0;
    for (int d = 0; d < count; ++d)
        if (probs[d].n < 1 || probs[d].m < 1) return 0;
    return plan_of(probs, count, o).total;
}

pc_status pc_corr(pc_ctx *ctx, const double *X, int64_t m, int64_t n, double alpha, void *ws,
                  size_t ws_bytes, void *C_out, uint64_t *adj_out) {
    if (!ctx || !X) return PC_ERR_INVALID_ARG;
    if (!(alpha > 0.0 && alpha < 1.0)) return PC_ERR_INVALID_ARG;
    pc_status s = check_shape(n, m);
    if (s != PC_OK) return s;
    const Plan L = make_plan(&n, &m, 1, ctx->opt);
    if ((s = check_ws(ws, ws_bytes, L)) != PC_OK) return s;
    if ((s = ensure_binom(ctx, n)) != PC_OK) return s;
    unsigned char *w = static_cast<unsigned char *>(ws);
    pc_problem p{};
    p.X = X;
    p.m = m;
    p.n = n;
    p.alpha = alpha;
    p.max_level = 0;
    std::vector<Prob> probs;
    fill_probs(ctx, L, w, &p, probs);
    if ((s = upload_table(ctx, L, w, probs)) != PC_OK) return s;
    const Batch b = make_batch(ctx, L, w);
    if ((s = enqueue_corr(ctx, b, L, false)) != PC_OK) return s;
    const size_t esz = ctx->opt.precision == PC_PREC_FP64 ? sizeof(double) : sizeof(float);
    if (C_out) PC_HIP(hipMemcpyAsync(C_out, w + L.reg[0].c, esz * n * n, hipMemcpyDeviceToDevice, ctx->stream));
    if (adj_out)
        PC_HIP(hipMemcpyAsync(adj_out, w + L.reg[0].adj, sizeof(uint64_t) * n * words_per_row(n),
                              hipMemcpyDeviceToDevice, ctx->stream));
    return PC_OK;
}

pc_status pc_sync_status(pc_ctx *ctx, void *ws, size_t ws_bytes) {
    if (!ctx) return PC_ERR_INVALID_ARG;
    PC_HIP(hipStreamSynchronize(ctx->stream));
    if (!ws) return PC_OK;
    const size_t table = align256(sizeof(DevState));
    if (ws_bytes < table + sizeof(Prob)) return PC_ERR_WORKSPACE;
    int err = 0;
    PC_HIP(hipMemcpy(&err, static_cast<unsigned char *>(ws) + table + offsetof(Prob, err), sizeof(int),
                     hipMemcpyDeviceToHost));
    return (pc_status)err;
}

}  // extern "C"

namespace {

// One caller-driven level (pc_level, pc_level_corr). C_given: a caller's FP64 correlation matrix,
// copied into the workspace first (then m_nominal sets the thresholds).
pc_status level_common(pc_ctx *ctx, int level, int64_t n, int64_t m, double alpha, uint64_t *adj,
                       const pc_sepset *sep, pc_run_stats *st, void *ws, size_t ws_bytes,
                       const double *C_given, double m_nominal) {
    if (!ctx || !adj || !sep || !sep->count || (!sep->recs && sep->cap > 0)) return PC_ERR_INVALID_ARG;
    if (level < 1 || level > PC_MAX_LEVEL) return PC_ERR_INVALID_ARG;
    if (!(alpha > 0.0 && alpha < 1.0)) return PC_ERR_INVALID_ARG;
    pc_status s = check_shape(n, m);
    if (s != PC_OK) return s;
    const Plan L = make_plan(&n, &m, 1, ctx->opt);
    if ((s = check_ws(ws, ws_bytes, L)) != PC_OK) return s;
    if ((s = ensure_binom(ctx, n)) != PC_OK) return s;
    const auto t0 = std::chrono::steady_clock::now();
    unsigned char *w = static_cast<unsigned char *>(ws);
    pc_problem p{};
    p.m = m;
    p.n = n;
    p.alpha = alpha;
    p.max_level = level;
    p.adj_out = adj;
    p.sep = *sep;
    std::vector<Prob> probs;
    fill_probs(ctx, L, w, &p, probs, m_nominal);
    if ((s = upload_table(ctx, L, w, probs)) != PC_OK) return s;
    if (C_given)
        PC_HIP(hipMemcpyAsync(w + L.reg[0].c, C_given, sizeof(double) * (size_t)n * (size_t)n,
                              hipMemcpyDeviceToDevice, ctx->stream));
    const Batch b = make_batch(ctx, L, w);
    reset_timed(ctx);
    PC_HIP(launch_rearm(ctx->stream, b));
    if ((s = enqueue_level(ctx, b, level, false)) != PC_OK) return s;
    std::vector<Prob> host;
    pc_status status = PC_OK;
    int promoted = 0;
    const pc_status r = collect_promoting(ctx, L, w, level, nullptr, &status, host, &promoted);
    if (r < 0 && r != PC_ERR_SEPSET_CAPACITY) return r;
    const Prob &P = host[0];
    if (st) {
        st->tests[level] = P.tests[level];
        st->removed[level] = P.removed[level];
        st->rechecks[level] = P.rechecks[level];
        st->items[level] = P.items[level];
        st->audit_violations[level] = P.audit_viol[level];
        st->max_degree[level] = P.maxdeg[level];
        st->fp64_from = promoted;
        const int tm = ctx->opt.timing;
        const unsigned long long bit = 1ull << level;
        if ((tm & 4) && (ctx->rec_compact & bit))
            st->compact_ms[level] = event_ms(ctx->ev_compact[level][0], ctx->ev_compact[level][1]);
        if ((tm & 2) && (ctx->rec_level & bit)) st->level_ms[level] = event_ms(ctx->ev_level[level][0], ctx->ev_level[level][1]);
        if ((tm & 8) && (ctx->rec_recheck & bit))
            st->recheck_ms[level] = event_ms(ctx->ev_recheck[level][0], ctx->ev_recheck[level][1]);
        st->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (r == PC_ERR_SEPSET_CAPACITY) return r;
    if (std::isnan(P.tau[level]) && P.maxdeg[level] >= level + 1) return PC_WARN_SAMPLE_LIMIT;
    return PC_OK;
}

// Sample count of the workspace plan of a given-C call (no data is stored).
constexpr int64_t kGivenPlanM = 4;

pc_status check_given(const pc_ctx *ctx, const double *C, double m) {
    if (!ctx || !C) return PC_ERR_INVALID_ARG;
    if (!(m > 0.0) || !std::isfinite(m)) return PC_ERR_INVALID_ARG;
    if (ctx->opt.precision != PC_PREC_FP64) return PC_ERR_UNSUPPORTED;
    return PC_OK;
}

}  // namespace

extern "C" {

pc_status pc_level(pc_ctx *ctx, int level, int64_t n, int64_t m, double alpha, uint64_t *adj,
                   const pc_sepset *sep, pc_run_stats *st, void *ws, size_t ws_bytes) {
    return level_common(ctx, level, n, m, alpha, adj, sep, st, ws, ws_bytes, nullptr, -1.0);
}

size_t pc_corr_workspace_bytes(int64_t n, const pc_options *opt) { return pc_workspace_bytes(n, kGivenPlanM, opt); }

pc_status pc_level_corr(pc_ctx *ctx, int level, const double *C, int64_t n, double m, double alpha,
                        uint64_t *adj, const pc_sepset *sep, pc_run_stats *st, void *ws, size_t ws_bytes) {
    pc_status s = check_given(ctx, C, m);
    if (s != PC_OK) return s;
    return level_common(ctx, level, n, kGivenPlanM, alpha, adj, sep, st, ws, ws_bytes, C, m);
}

pc_status pc_skeleton_corr(pc_ctx *ctx, const double *C, int64_t n, double m, double alpha, int max_level,
                           uint64_t *adj_out, const pc_sepset *sep, pc_run_stats *st, void *ws, size_t ws_bytes) {
    pc_status s = check_given(ctx, C, m);
    if (s != PC_OK) return s;
    if (!adj_out || !sep || !sep->count || (!sep->recs && sep->cap > 0)) return PC_ERR_INVALID_ARG;
    if (!(alpha > 0.0 && alpha < 1.0)) return PC_ERR_INVALID_ARG;
    if ((s = check_shape(n, kGivenPlanM)) != PC_OK) return s;
    const auto t0 = std::chrono::steady_clock::now();
    int64_t mp = kGivenPlanM;
    const Plan L = make_plan(&n, &mp, 1, ctx->opt);
    if ((s = check_ws(ws, ws_bytes, L)) != PC_OK) return s;
    if ((s = ensure_binom(ctx, n)) != PC_OK) return s;
    unsigned char *w = static_cast<unsigned char *>(ws);
    pc_problem p{};
    p.m = kGivenPlanM;
    p.n = n;
    p.alpha = alpha;
    p.max_level = max_level;
    p.adj_out = adj_out;
    p.sep = *sep;
    std::vector<Prob> table;
    fill_probs(ctx, L, w, &p, table, m);
    if ((s = upload_table(ctx, L, w, table)) != PC_OK) return s;
    PC_HIP(hipMemcpyAsync(w + L.reg[0].c, C, sizeof(double) * (size_t)n * (size_t)n, hipMemcpyDeviceToDevice,
                          ctx->stream));
    if ((s = enqueue_skeletons(ctx, &p, 1, L, w, false, nullptr, true)) != PC_OK) return s;
    std::vector<Prob> host;
    pc_status status = PC_OK;
    const pc_status r = collect(ctx, L.table, L.st, 1, w, st, &status, host);
    if (r == PC_ERR_HIP) return r;
    if (st) {
        fill_times(ctx, st, ctx->top_run);
        st->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

pc_status pc_skeleton(pc_ctx *ctx, const double *X, int64_t m, int64_t n, double alpha,
                      int max_level, uint64_t *adj_out, const pc_sepset *sep, pc_run_stats *st,
                      void *ws, size_t ws_bytes) {
    if (!ctx || !sep) return PC_ERR_INVALID_ARG;
    pc_problem p{};
    p.X = X;
    p.m = m;
    p.n = n;
    p.alpha = alpha;
    p.max_level = max_level;
    p.adj_out = adj_out;
    p.sep = *sep;
    const auto t0 = std::chrono::steady_clock::now();
    Plan L;
    std::vector<Prob> table;
    pc_status s = prepare(ctx, &p, 1, ws, ws_bytes, L, table);
    if (s != PC_OK) return s;
    unsigned char *w = static_cast<unsigned char *>(ws);
    if ((s = enqueue_skeletons(ctx, &p, 1, L, w, false)) != PC_OK) return s;
    std::vector<Prob> host;
    pc_status status = PC_OK;
    const pc_status r = collect_promoting(ctx, L, w, levels_to_enqueue(&p, 1), st, &status, host);
    if (r == PC_ERR_HIP) return r;
    if (st) {
        fill_times(ctx, st, ctx->top_run);
        st->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

pc_status pc_skeleton_noalloc(pc_ctx *ctx, const double *X, int64_t m, int64_t n, double alpha, int max_level,
                              uint64_t *adj_out, const pc_sepset *sep, pc_run_stats *st) {
    if (!ctx || !sep) return PC_ERR_INVALID_ARG;
    if (!ctx->scratch) return PC_ERR_HIP;
    pc_status s = check_shape(n, m);
    if (s != PC_OK) return s;
    // Everything pc_skeleton would allocate must already exist: the workspace fits the array, the
    // binomial table covers n, the problem table fits the pinned staging.
    const Plan L = make_plan(&n, &m, 1, ctx->opt);
    if (L.total > (size_t)PC_NOALLOC_SCRATCH_BYTES || n + 1 > ctx->binom_rows || L.table_bytes > ctx->staging_bytes)
        return PC_ERR_WORKSPACE;
    return pc_skeleton(ctx, X, m, n, alpha, max_level, adj_out, sep, st, ctx->scratch, PC_NOALLOC_SCRATCH_BYTES);
}

pc_status pc_batch_skeleton(pc_ctx *ctx, const pc_problem *probs, int count, pc_run_stats *st,
                            pc_status *status, void *ws, size_t ws_bytes) {
    if (!ctx || !probs || count < 1) return PC_ERR_INVALID_ARG;
    const auto t0 = std::chrono::steady_clock::now();
    Plan L;
    std::vector<Prob> table;
    pc_status s = prepare(ctx, probs, count, ws, ws_bytes, L, table);
    if (s != PC_OK) return s;
    unsigned char *w = static_cast<unsigned char *>(ws);
    if ((s = enqueue_skeletons(ctx, probs, count, L, w, false)) != PC_OK) return s;
    std::vector<Prob> host;
    const pc_status r = collect_promoting(ctx, L, w, levels_to_enqueue(probs, count), st, status, host);
    if (st) {
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (int d = 0; d < count; ++d) {
            fill_times(ctx, &st[d], ctx->top_run);   // the phases are timed per launch: the batch's
            st[d].wall_ms = ms;
        }
    }
    return r;
}

pc_status pc_batch_capture(pc_ctx *ctx, const pc_problem *probs, int count, void *ws,
                           size_t ws_bytes, pc_graph **out) {
    return pc_batch_capture_ordered(ctx, probs, count, nullptr, ws, ws_bytes, out);
}

pc_status pc_batch_capture_ordered(pc_ctx *ctx, const pc_problem *probs, int count, const pc_order *order, void *ws,
                                   size_t ws_bytes, pc_graph **out) {
    if (!ctx || !probs || count < 1 || !out) return PC_ERR_INVALID_ARG;
    if (order && !valid_order(order)) return PC_ERR_INVALID_ARG;
    *out = nullptr;
    if (ctx->stream == nullptr) return PC_ERR_INVALID_ARG;  // the null stream cannot be captured
    Plan L;
    pc_graph *g = new (std::nothrow) pc_graph();
    if (!g) return PC_ERR_HIP;
    pc_status s = prepare(ctx, probs, count, ws, ws_bytes, L, g->host_probs);
    if (s != PC_OK) { delete g; return s; }
    g->ctx = ctx;
    g->ws = static_cast<unsigned char *>(ws);
    g->count = count;
    g->table_off = L.table;
    g->st_off = L.st;
    g->probs.assign(probs, probs + count);
    g->top = levels_to_enqueue(probs, count);
    g->captured = std::min(g->top, graph_levels_of(ctx->opt));
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) { delete g; return PC_ERR_HIP; }
    if (hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        delete g;
        return PC_ERR_HIP;
    }
    g->has_order = order != nullptr;
    if (order) g->order = *order;
    s = enqueue_skeletons(ctx, probs, count, L, g->ws, true, order);
    g->tail = ctx->tail_enqueued;
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(ctx->stream, &graph);
    if (s != PC_OK || ec != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        delete g;
        return s != PC_OK ? s : PC_ERR_HIP;
    }
    g->graph = graph;
    if (hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        delete g;
        return PC_ERR_HIP;
    }
    *out = g;
    return PC_OK;
}

pc_status pc_graph_launch(pc_graph *g) {
    if (!g) return PC_ERR_INVALID_ARG;
    PC_HIP(hipGraphLaunch(g->exec, g->ctx->stream));
    return PC_OK;
}

pc_status pc_graph_results(pc_graph *g, pc_run_stats *st, pc_status *status) {
    if (!g) return PC_ERR_INVALID_ARG;
    pc_ctx *ctx = g->ctx;
    if (g->captured < g->top) {
        // Datasets that still have work after the recorded levels continue on the stream.
        const Plan L = plan_of(g->probs.data(), g->count, ctx->opt);
        const Batch b = make_batch(ctx, L, g->ws);
        int from = g->captured + 1;
        if (g->tail) {
            // after the tail kernel: from the smallest level it left to the level kernels
            std::vector<Prob> host;
            DevState ds;
            pc_status s = read_table(ctx, L, g->ws, host, ds);
            if (s != PC_OK) return s;
            from = 0;
            for (const Prob &P : host)
                if (P.tail_next > 0) from = from == 0 ? P.tail_next : std::min(from, P.tail_next);
            if (from > 0 && from <= g->top && !ds.done && (s = enqueue_plan(ctx, b, from, false)) != PC_OK) return s;
        }
        if (from > 0 && from <= g->top) {
            const OrderRun ord{&g->order, &L, g->ws};
            pc_status s = run_levels_eager(ctx, b, L, g->ws, from, g->top, g->has_order ? &ord : nullptr);
            if (s != PC_OK) return s;
        }
    }
    std::vector<Prob> host;
    const Plan L = plan_of(g->probs.data(), g->count, ctx->opt);
    return collect_promoting(ctx, L, g->ws, g->top, st, status, host);
}

void pc_graph_destroy(pc_graph *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

size_t pc_ordered_workspace_bytes(int64_t n, int64_t m, const pc_options *opt, const pc_order *order) {
    if (!valid_order(order)) return 0;
    return pc_workspace_bytes(n, m, opt);
}

pc_status pc_skeleton_ordered(pc_ctx *ctx, const double *X, int64_t m, int64_t n, double alpha,
                              int max_level, const pc_order *order, uint64_t *adj_out,
                              const pc_sepset *sep, pc_run_stats *st, void *ws, size_t ws_bytes) {
    if (!ctx || !sep || !valid_order(order)) return PC_ERR_INVALID_ARG;
    pc_problem p{};
    p.X = X;
    p.m = m;
    p.n = n;
    p.alpha = alpha;
    p.max_level = max_level;
    p.adj_out = adj_out;
    p.sep = *sep;
    pc_status s = check_problem(p);
    if (s != PC_OK) return s;
    const Plan L = make_plan(&n, &m, 1, ctx->opt);
    if ((s = check_ws(ws, ws_bytes, L)) != PC_OK) return s;
    if ((s = ensure_binom(ctx, n)) != PC_OK) return s;
    const auto t0 = std::chrono::steady_clock::now();
    unsigned char *w = static_cast<unsigned char *>(ws);
    std::vector<Prob> table;
    fill_probs(ctx, L, w, &p, table);
    if ((s = upload_table(ctx, L, w, table)) != PC_OK) return s;
    if ((s = enqueue_skeletons(ctx, &p, 1, L, w, false, order)) != PC_OK) return s;
    std::vector<Prob> host;
    pc_status status = PC_OK;
    const pc_status r = collect_promoting(ctx, L, w, levels_to_enqueue(&p, 1), st, &status, host);
    if (r == PC_ERR_HIP) return r;
    if (st) {
        fill_times(ctx, st, ctx->top_run);
        st->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

namespace {

// Common part of the feature calls: the snapshot copied into the workspace, the problem table of
// the level, and G' compacted from the snapshot.
pc_status features_setup(pc_ctx *ctx, int level, int64_t n, int64_t m, double alpha, const uint64_t *adj, void *ws,
                         size_t ws_bytes, Plan &L, Batch &b) {
    if (level < 1 || level > PC_MAX_LEVEL || !(alpha > 0.0 && alpha < 1.0)) return PC_ERR_INVALID_ARG;
    pc_status s = check_shape(n, m);
    if (s != PC_OK) return s;
    L = make_plan(&n, &m, 1, ctx->opt);
    if ((s = check_ws(ws, ws_bytes, L)) != PC_OK) return s;
    if ((s = ensure_binom(ctx, n)) != PC_OK) return s;
    unsigned char *w = static_cast<unsigned char *>(ws);
    // The snapshot is copied into the workspace's own bit matrix, so the caller's stays untouched.
    PC_HIP(hipMemcpyAsync(w + L.reg[0].adj, adj, sizeof(uint64_t) * n * words_per_row(n), hipMemcpyDeviceToDevice,
                          ctx->stream));
    pc_problem p{};
    p.m = m;
    p.n = n;
    p.alpha = alpha;
    p.max_level = level;
    std::vector<Prob> probs;
    fill_probs(ctx, L, w, &p, probs);
    if ((s = upload_table(ctx, L, w, probs)) != PC_OK) return s;
    b = make_batch(ctx, L, w);
    PC_HIP(launch_rearm(ctx->stream, b));
    PC_HIP(launch_compact(ctx->stream, b, level, ranks_per_item(ctx, level)));
    return PC_OK;
}

// Reads the feature row count (the last entry of the row offsets) and synchronises.
pc_status feature_rows(pc_ctx *ctx, const long long *foff, long long total_rows, int64_t cap, int64_t *rows_out) {
    long long rows = 0;
    PC_HIP(hipMemcpyAsync(&rows, foff + total_rows, sizeof(rows), hipMemcpyDeviceToHost, ctx->stream));
    PC_HIP(hipStreamSynchronize(ctx->stream));
    *rows_out = rows;
    return rows > cap ? PC_ERR_WORKSPACE : PC_OK;
}

}  // namespace

pc_status pc_features(pc_ctx *ctx, int level, int64_t n, int64_t m, double alpha, const uint64_t *adj,
                      float *feats, int32_t *meta, int64_t cap, int64_t *rows_out, void *ws,
                      size_t ws_bytes) {
    if (!ctx || !adj || !feats || !rows_out || cap < 0) return PC_ERR_INVALID_ARG;
    Plan L;
    Batch b;
    pc_status s = features_setup(ctx, level, n, m, alpha, adj, ws, ws_bytes, L, b);
    if (s != PC_OK) return s;
    unsigned char *w = static_cast<unsigned char *>(ws);
    // Feature offsets go to the level's item-offset buffer (free until the level runs).
    long long *foff = reinterpret_cast<long long *>(w + L.item_off);
    int *skip = reinterpret_cast<int *>(w + L.nitems);
    PC_HIP(launch_feat_plan(ctx->stream, b, foff, cap, skip));
    PC_HIP(launch_features(ctx->stream, b, level, foff, feats, meta, skip));
    return feature_rows(ctx, foff, L.total_rows, cap, rows_out);
}

pc_status pc_row_features(pc_ctx *ctx, int level, int64_t n, int64_t m, double alpha, const uint64_t *adj,
                          float *feats, float *labels, int32_t *meta, int64_t cap, int64_t *rows_out,
                          void *ws, size_t ws_bytes) {
    if (!ctx || !adj || !feats || !labels || !rows_out || cap < 0 || level != 1) return PC_ERR_INVALID_ARG;
    Plan L;
    Batch b;
    pc_status s = features_setup(ctx, level, n, m, alpha, adj, ws, ws_bytes, L, b);
    if (s != PC_OK) return s;
    unsigned char *w = static_cast<unsigned char *>(ws);
    long long *foff = reinterpret_cast<long long *>(w + L.item_off);
    int *skip = reinterpret_cast<int *>(w + L.nitems);
    PC_HIP(launch_row_features(ctx->stream, b, level, foff, cap, skip, feats, labels, meta));
    return feature_rows(ctx, foff, L.total_rows, cap, rows_out);
}

pc_status pc_row_scores(pc_ctx *ctx, int64_t n, int64_t m, double alpha, const uint64_t *adj, const pc_order *order,
                        float *scores, int32_t *top, void *ws, size_t ws_bytes) {
    if (!ctx || !adj || !scores || !top || !order) return PC_ERR_INVALID_ARG;
    if (!row_order_on(order) || !valid_order(order)) return PC_ERR_INVALID_ARG;
    Plan L;
    Batch b;
    pc_status s = features_setup(ctx, 1, n, m, alpha, adj, ws, ws_bytes, L, b);
    if (s != PC_OK) return s;
    PC_HIP(launch_row_order(ctx->stream, b, 1, order->row_params, order->row_top, order->row_rank, order->row_short,
                            order->row_sort, ctx->num_cu, scores, top));
    PC_HIP(hipStreamSynchronize(ctx->stream));
    return PC_OK;
}

pc_status pc_mlp_forward(pc_ctx *ctx, const float *params, const float *X, int64_t rows, float *scores,
                         float *act) {
    if (!ctx || !params || !X || !scores || rows < 0) return PC_ERR_INVALID_ARG;
    if (rows == 0) return PC_OK;
    const long long tiles = (rows + 63) / 64;
    const int grid = (int)std::min<long long>(tiles, 8LL * ctx->num_cu);
    PC_HIP(launch_mlp_forward(ctx->stream, params, X, rows, nullptr, rows, scores, act, nullptr, grid));
    return PC_OK;
}

pc_status pc_mlp_backward(pc_ctx *ctx, const float *params, const float *X, int64_t rows, const float *act,
                          const float *dscore, float *grads, float *partial) {
    if (!ctx || !params || !X || !act || !dscore || !grads || !partial || rows <= 0) return PC_ERR_INVALID_ARG;
    PC_HIP(launch_mlp_backward(ctx->stream, params, X, rows, act, dscore, partial, grads));
    return PC_OK;
}

pc_status pc_mlp_bce(pc_ctx *ctx, const float *scores, const float *labels, int64_t rows, float pos_weight,
                     float *dscore, double *loss) {
    if (!ctx || !scores || !labels || !dscore || !loss || rows <= 0) return PC_ERR_INVALID_ARG;
    PC_HIP(launch_bce(ctx->stream, scores, labels, rows, pos_weight, dscore, loss));
    return PC_OK;
}

pc_status pc_mlp_adam(pc_ctx *ctx, float *params, const float *grads, float *m1, float *m2, int step,
                      float lr, float beta1, float beta2, float eps) {
    if (!ctx || !params || !grads || !m1 || !m2 || step < 1) return PC_ERR_INVALID_ARG;
    PC_HIP(launch_adam(ctx->stream, params, grads, m1, m2, step, lr, beta1, beta2, eps));
    return PC_OK;
}

// Orientation workspace: IN, two proposal buffers (n x W words each), the SepSet index (n x n
// int32) and the round counter.
size_t orient_ws_bytes(int64_t n) {
    const size_t bits = align256((size_t)n * (size_t)words_per_row(n) * sizeof(uint64_t));
    return 3 * bits + align256((size_t)n * (size_t)n * sizeof(int)) + 256;
}

size_t pc_orient_workspace_bytes(int64_t n) {
    if (check_shape(n, 4) != PC_OK) return 0;
    return orient_ws_bytes(n);
}

pc_status pc_orient(pc_ctx *ctx, int64_t n, const uint64_t *adj, const pc_sep_rec *recs, int64_t nrec,
                    uint64_t *arrows, void *ws, size_t ws_bytes, int32_t *rounds) {
    if (!ctx || !adj || !arrows || !ws || nrec < 0 || (nrec > 0 && !recs)) return PC_ERR_INVALID_ARG;
    pc_status st = check_shape(n, 4);
    if (st != PC_OK) return st;
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return PC_ERR_INVALID_ARG;
    if (ws_bytes < orient_ws_bytes(n)) return PC_ERR_WORKSPACE;
    const size_t bits = align256((size_t)n * (size_t)words_per_row(n) * sizeof(uint64_t));
    unsigned char *w = static_cast<unsigned char *>(ws);
    auto *IN = reinterpret_cast<unsigned long long *>(w);
    auto *P0 = reinterpret_cast<unsigned long long *>(w + bits);
    auto *P1 = reinterpret_cast<unsigned long long *>(w + 2 * bits);
    int *sep_idx = reinterpret_cast<int *>(w + 3 * bits);
    int *flag = reinterpret_cast<int *>(w + 3 * bits + align256((size_t)n * (size_t)n * sizeof(int)));
    const auto *A = reinterpret_cast<const unsigned long long *>(adj);
    auto *OUT = reinterpret_cast<unsigned long long *>(arrows);
    hipStream_t s = ctx->stream;
    PC_HIP(launch_orient_setup(s, n, A, recs, nrec, OUT, IN, P0, P1, sep_idx, flag));
    // Every round that changes something orients at least one of the n(n-1)/2 possible edges.
    int32_t done = 0;
    for (int64_t r = 0; r <= n * (n - 1) / 2; ++r) {
        PC_HIP(launch_orient_round(s, n, A, OUT, IN, (r & 1) ? P1 : P0, (r & 1) ? P0 : P1, flag));
        int changed = 0;
        PC_HIP(hipMemcpyAsync(&changed, flag, sizeof(int), hipMemcpyDeviceToHost, s));
        PC_HIP(hipStreamSynchronize(s));
        if (changed == 0) break;
        ++done;
    }
    if (rounds) *rounds = done;
    return PC_OK;
}

pc_status pc_comb_unrank(int32_t d, int32_t l, uint64_t t, int32_t skip, int32_t *out) {
    if (!out || d < 0 || l < 0 || l > PC_MAX_LEVEL) return PC_ERR_INVALID_ARG;
    const int pool = skip >= 0 ? d - 1 : d;
    if (skip >= d || pool < l) return PC_ERR_INVALID_ARG;
    auto binom = [](int a, int b) -> unsigned long long {
        if (b < 0 || a < b) return 0ull;
        unsigned long long c = 1;
        for (int k = 0; k < b; ++k) c = c * (unsigned long long)(a - k) / (unsigned long long)(k + 1);
        return c;
    };
    if (t >= binom(pool, l)) return PC_ERR_INVALID_ARG;
    int P[PC_MAX_LEVEL];
    // Dispatch on the compile-time subset size the device code uses.
    static_assert(PC_MAX_LEVEL == 30, "one case per subset size up to PC_MAX_LEVEL");
    switch (l) {
        case 0: break;
#define PC_CASE(K)                                                        \
    case K: {                                                             \
        int Q[K];                                                         \
        comb_unrank<K>(pool, t, Q, binom);                                \
        for (int c = 0; c < K; ++c) P[c] = Q[c];                          \
        break;                                                            \
    }
        PC_CASE(1) PC_CASE(2) PC_CASE(3) PC_CASE(4) PC_CASE(5) PC_CASE(6) PC_CASE(7)
        PC_CASE(8) PC_CASE(9) PC_CASE(10) PC_CASE(11) PC_CASE(12) PC_CASE(13) PC_CASE(14)
        PC_CASE(15) PC_CASE(16) PC_CASE(17) PC_CASE(18) PC_CASE(19) PC_CASE(20) PC_CASE(21)
        PC_CASE(22) PC_CASE(23) PC_CASE(24) PC_CASE(25) PC_CASE(26) PC_CASE(27) PC_CASE(28)
        PC_CASE(29) PC_CASE(30)
#undef PC_CASE
        default: return PC_ERR_INVALID_ARG;
    }
    for (int c = 0; c < l; ++c) out[c] = (skip >= 0 && P[c] >= skip) ? P[c] + 1 : P[c];
    return PC_OK;
}

double pc_threshold(double alpha, double m, int level) {
    if (!(alpha > 0.0 && alpha < 1.0)) return NAN;
    return tau_of(z_of_alpha(alpha), m, level);
}

pc_status pc_set_tuning(pc_ctx *ctx, const pc_tuning *t) {
    if (!ctx) return PC_ERR_INVALID_ARG;
    if (!t) {
        ctx->tuned = false;
        return PC_OK;
    }
    for (int l = 0; l <= PC_MAX_LEVEL; ++l)
        if (t->tests_per_lane[l] < 0 || t->ranks_per_lane[l] < 0 || t->ranks_per_lane[l] > 64 ||
            t->lds_budget[l] < -1 || t->grid[l] < 0 || t->grid[l] > (1 << 20) || t->recheck_grid[l] < 0 ||
            t->recheck_grid[l] > (1 << 20) ||
            (t->set_lanes[l] != 0 && (t->set_lanes[l] < 4 || t->set_lanes[l] > 64 ||
                                      (t->set_lanes[l] & (t->set_lanes[l] - 1)) != 0)))
            return PC_ERR_INVALID_ARG;
    ctx->tuning = *t;
    ctx->tuned = true;
    return PC_OK;
}

// Coordinate search over the level kernels' shapes: each pass varies one parameter for every
// level at once, and each level keeps its fastest value (levels are timed independently: the
// skeleton, and so the work of every level, does not depend on the shapes).
pc_status pc_tune(pc_ctx *ctx, const pc_problem *probs, int count, const pc_order *order, void *ws,
                  size_t ws_bytes, pc_tuning *out) {
    if (!ctx || !probs || count < 1 || !out || (order && count != 1)) return PC_ERR_INVALID_ARG;
    constexpr int NL = PC_MAX_LEVEL + 1;
    const int saved_timing = ctx->opt.timing;
    const bool saved_tuned = ctx->tuned;
    const pc_tuning saved = ctx->tuning;
    std::vector<pc_run_stats> st((size_t)count);
    std::vector<pc_status> status((size_t)count);
    int levels = 0, runs = 0;
    ctx->opt.timing = 2 | 8;   // the level and re-check kernels, HIP events around each
    auto run = [&](const pc_tuning &t, float (&ms)[NL], double (&tests)[NL]) -> pc_status {
        ctx->tuning = t;
        ctx->tuned = true;
        for (float &x : ms) x = INFINITY;
        for (double &x : tests) x = INFINITY;
        for (int rep = 0; rep < 2; ++rep) {
            pc_status r;
            if (order) {
                const pc_problem &p = probs[0];
                r = pc_skeleton_ordered(ctx, p.X, p.m, p.n, p.alpha, p.max_level, order, p.adj_out, &p.sep,
                                        st.data(), ws, ws_bytes);
            } else {
                r = pc_batch_skeleton(ctx, probs, count, st.data(), status.data(), ws, ws_bytes);
            }
            ++runs;
            if (r < 0) return r;
            int lr = st[0].levels_run;
            if (!order)
                for (int d = 1; d < count; ++d) lr = std::max(lr, st[d].levels_run);
            levels = std::max(levels, lr);
            for (int l = 1; l < std::min(lr, NL); ++l) {
                if (st[0].level_ms[l] > 0.f) ms[l] = std::min(ms[l], st[0].level_ms[l] + st[0].recheck_ms[l]);
                double tl = 0.0;
                for (int d = 0; d < (order ? 1 : count); ++d) tl += (double)st[d].tests[l];
                tests[l] = std::min(tests[l], tl);
            }
        }
        return PC_OK;
    };
    pc_tuning cur{};
    for (int l = 0; l < NL; ++l) cur.lds_budget[l] = -1;
    float base[NL], best[NL], fastest[NL], ms[NL];
    double base_tests[NL], best_tests[NL], tests[NL];
    pc_status r = run(cur, base, base_tests);
    for (int l = 0; l < NL; ++l) {
        best[l] = fastest[l] = base[l];
        best_tests[l] = base_tests[l];
    }
    // One pass: every level tries each value of one field and keeps a value that is at least 1%
    // faster than its current one, or within 2% of the fastest time seen at that level while
    // running at least 10% fewer CI tests (latency-bound launches take about as long with more
    // speculative tests; the shape that wastes fewer of them is kept).
    auto pass = [&](int32_t (pc_tuning::*field)[NL], std::initializer_list<int> values, int from_level,
                    int to_level) {
        pc_tuning next = cur;
        for (int v : values) {
            if (r < 0) return;
            pc_tuning t = cur;
            for (int l = from_level; l <= to_level; ++l) (t.*field)[l] = v;
            if ((r = run(t, ms, tests)) < 0) return;
            for (int l = from_level; l <= to_level; ++l) {
                const bool faster = ms[l] < 0.99f * best[l];
                const bool leaner = ms[l] <= 1.02f * fastest[l] && tests[l] <= 0.9 * best_tests[l];
                fastest[l] = std::min(fastest[l], ms[l]);
                if (faster || leaner) {
                    best[l] = ms[l];
                    best_tests[l] = tests[l];
                    (next.*field)[l] = v;
                }
            }
        }
        cur = next;
    };
    if (r >= 0) pass(&pc_tuning::tests_per_lane, {16, 32, 64, 128, 256, 512, 1024, 2048}, 1, NL - 1);
    if (r >= 0) pass(&pc_tuning::lds_budget, {0, 8192, 16384, 32768}, 1, NL - 1);
    if (r >= 0) pass(&pc_tuning::ranks_per_lane, {1, 2, 4, 8}, 1, NL - 1);
    if (r >= 0) pass(&pc_tuning::set_lanes, {16, 64}, 1, kWaveSetLevels);
    if (r >= 0) pass(&pc_tuning::grid, {16, 64, 256}, 1, NL - 1);
    if (r >= 0) pass(&pc_tuning::recheck_grid, {16, 64, 256}, 1, NL - 1);
    ctx->opt.timing = saved_timing;
    if (r < 0) {
        ctx->tuning = saved;
        ctx->tuned = saved_tuned;
        return r;
    }
    for (int l = 0; l < NL; ++l) {
        cur.level_ms[l] = std::isfinite(best[l]) ? best[l] : 0.f;
        cur.default_ms[l] = std::isfinite(base[l]) ? base[l] : 0.f;
    }
    cur.levels = levels;
    cur.runs = runs;
    *out = cur;
    ctx->tuning = cur;
    ctx->tuned = true;
    return PC_OK;
}

size_t pc_abi_size(int which) {
    switch (which) {
        case 0: return sizeof(pc_options);
        case 1: return sizeof(pc_sep_rec);
        case 2: return sizeof(pc_sepset);
        case 3: return sizeof(pc_run_stats);
        case 4: return sizeof(pc_problem);
        case 5: return sizeof(pc_order);
        case 6: return sizeof(pc_tuning);
        default: return 0;
    }
}

const char *pc_status_str(pc_status s) {
    switch (s) {
        case PC_OK: return "ok";
        case PC_WARN_SAMPLE_LIMIT: return "stopped: m - level - 3 <= 0";
        case PC_WARN_LEVEL_CAP: return "stopped at the largest supported level";
        case PC_ERR_INVALID_ARG: return "invalid argument";
        case PC_ERR_SHAPE: return "invalid shape";
        case PC_ERR_CONSTANT_COLUMN: return "a variable has zero variance";
        case PC_ERR_NONFINITE: return "data holds NaN or Inf";
        case PC_ERR_WORKSPACE: return "workspace or re-check queue too small";
        case PC_ERR_HIP: return "HIP runtime error";
        case PC_ERR_UNSUPPORTED: return "unsupported device or work count";
        case PC_ERR_SEPSET_CAPACITY: return "SepSet table too small";
    }
    return "unknown status";
}

}  // extern "C"
