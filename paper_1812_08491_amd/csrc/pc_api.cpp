// C ABI of libpc.so: argument checks, workspace planning and the host level loop (Algorithm 2).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "pc.h"
#include "pc_comb.h"
#include "pc_dev.h"

using namespace pcg;

struct pc_ctx {
    hipStream_t stream;
    pc_options opt;
    int device;
    int num_cu;
    DevState *host_state;   // pinned, read back after each level
    hipEvent_t ev[2 * (PC_MAX_LEVEL + 2) + 2];
};

namespace {

constexpr double kU32 = 5.9604644775390625e-08;  // 2^-24, unit roundoff of FP32

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
    o.lds_budget = 65536;
    o.ranks_per_lane = 0;
    o.grid = 0;
    o.timing = 0;
    o.recheck_cap = 0;
    return o;
}

bool valid_options(const pc_options &o) {
    if (o.precision < PC_PREC_FP64 || o.precision > PC_PREC_BF16X3) return false;
    if (!(o.margin_scale >= 1.0f)) return false;
    if (o.lds_budget < 0 || o.ranks_per_lane < 0 || o.grid < 0 || o.recheck_cap < 0) return false;
    return true;
}

int64_t rq_cap_of(const pc_options &o) { return o.recheck_cap > 0 ? o.recheck_cap : (int64_t)1 << 20; }

// Standard normal CDF from erfc, and its inverse by Halley's method started from the rational
// approximation of Abramowitz & Stegun 26.2.23 (|error| < 4.5e-4); three Halley steps reach full
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
double eps_c_of(int prec, int64_t mp) {
    if (prec == PC_PREC_FP32) return ((double)mp + 4.0) * kU32;
    if (prec == PC_PREC_BF16X3) return 3.0 * std::ldexp(1.0, -18) + (3.0 * (double)mp + 8.0) * kU32;
    return 0.0;
}

struct Ws {
    Layout L;
    unsigned char *base;
    DevState *st() const { return reinterpret_cast<DevState *>(base + L.state); }
    template <typename T> T *at(size_t off) const { return reinterpret_cast<T *>(base + off); }
};

pc_status check_ws(const pc_ctx *ctx, int64_t n, int64_t m, void *ws, size_t ws_bytes, Ws &out) {
    if (!ws) return PC_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return PC_ERR_INVALID_ARG;
    out.L = Layout::make(n, m, ctx->opt.precision, rq_cap_of(ctx->opt));
    if (ws_bytes < out.L.total) return PC_ERR_WORKSPACE;
    out.base = static_cast<unsigned char *>(ws);
    return PC_OK;
}

pc_status check_shape(int64_t n, int64_t m) {
    if (n < 2 || m < 4) return PC_ERR_SHAPE;
    if (n > (int64_t)1 << 20 || m > (int64_t)1 << 28) return PC_ERR_SHAPE;
    return PC_OK;
}

int auto_grid(const pc_ctx *ctx) { return ctx->opt.grid > 0 ? ctx->opt.grid : 2 * ctx->num_cu; }

int ranks_per_item(const pc_ctx *ctx, int level) {
    const int q = ctx->opt.ranks_per_lane > 0 ? ctx->opt.ranks_per_lane : (level == 1 ? 1 : 4);
    return q * kLevelThreads;
}

int level_lds_bytes(const pc_ctx *ctx) {
    const size_t fixed = level_lds_fixed(ctx->opt.precision);
    size_t budget = (size_t)ctx->opt.lds_budget;
    const size_t limit = 64 * 1024 - 1024 - fixed;  // stay within 64 KiB of dynamic LDS
    if (budget > limit) budget = limit;
    return (int)(fixed + budget);
}

// Correlation + level 0 into adjacency `adj`.
pc_status corr_impl(pc_ctx *ctx, const double *X, int64_t m, int64_t n, double alpha,
                    const Ws &w, unsigned long long *adj, long long *zero_count) {
    hipStream_t s = ctx->stream;
    const Layout &L = w.L;
    const int prec = ctx->opt.precision;
    PC_HIP(launch_init(s, w.st(), w.at<unsigned long long>(L.binom), n, zero_count));
    PC_HIP(launch_colstats(s, X, m, n, w.at<double>(L.mu), w.at<double>(L.inv), w.st()));
    PC_HIP(launch_standardize(s, X, m, n, L.mp, w.at<double>(L.mu), w.at<double>(L.inv),
                              w.at<double>(L.zt64), w.base + L.zlo, w.base + L.zhi, prec));
    CorrArgs a{};
    a.zt64 = w.at<double>(L.zt64);
    a.za = prec == PC_PREC_BF16X3 ? (const void *)(w.base + L.zhi) : (const void *)(w.base + L.zlo);
    a.zb = w.base + L.zlo;
    a.C = w.base + L.c;
    a.adj = adj;
    a.st = w.st();
    a.n = n;
    a.m = m;
    a.mp = L.mp;
    a.W = words_per_row(n);
    const double z = z_of_alpha(alpha);
    a.tau0 = tau_of(z, (double)m, 0);
    a.t0 = std::tanh(a.tau0);
    a.eps_c = eps_c_of(prec, L.mp);
    a.force_recheck = ctx->opt.force_recheck_all;
    PC_HIP(launch_corr(s, a, prec));
    return PC_OK;
}

// Launches compaction, the level kernel and the re-check of one level (no synchronisation).
pc_status level_launch(pc_ctx *ctx, int level, int64_t n, int64_t m, double alpha, const Ws &w,
                       unsigned long long *adj, const pc_sepset *sep, bool run_tests,
                       hipEvent_t e0, hipEvent_t e1, hipEvent_t e2) {
    hipStream_t s = ctx->stream;
    const Layout &L = w.L;
    const int prec = ctx->opt.precision;
    const int64_t W = words_per_row(n);
    const int R = ranks_per_item(ctx, level);
    if (e0) PC_HIP(hipEventRecord(e0, s));
    PC_HIP(launch_compact(s, adj, n, W, level, R, w.at<int>(L.nbr), w.at<int>(L.deg),
                          w.at<long long>(L.nitems), w.at<long long>(L.item_off),
                          w.at<unsigned long long>(L.binom), w.st()));
    if (e1) PC_HIP(hipEventRecord(e1, s));
    if (!run_tests) return PC_OK;
    const double z = z_of_alpha(alpha);
    const double tau = tau_of(z, (double)m, level);
    LevelArgs a{};
    a.C = w.base + L.c;
    a.zt64 = w.at<double>(L.zt64);
    a.adj = adj;
    a.nbr = w.at<int>(L.nbr);
    a.deg = w.at<int>(L.deg);
    a.item_off = w.at<long long>(L.item_off);
    a.binom = w.at<unsigned long long>(L.binom);
    a.st = w.st();
    a.recs = sep->recs;
    a.rec_count = reinterpret_cast<long long *>(sep->count);
    a.rec_cap = sep->cap;
    a.n = n;
    a.m = m;
    a.mp = L.mp;
    a.W = W;
    a.level = level;
    a.ranks_per_item = R;
    a.lds_bytes = level_lds_bytes(ctx);
    a.force_recheck = prec != PC_PREC_FP64 && ctx->opt.force_recheck_all;
    a.tau = tau;
    a.t = (float)std::tanh(tau);
    const double eps = eps_c_of(prec, L.mp) + (4.0 * level + 16.0) * kU32;
    a.band = (float)((double)ctx->opt.margin_scale * eps);
    a.rq = w.at<pc_sep_rec>(L.rq);
    a.rq_cap = L.rq_cap;
    PC_HIP(launch_level(s, a, prec, auto_grid(ctx)));
    RecheckArgs r{};
    r.zt64 = prec == PC_PREC_FP64 ? nullptr : w.at<double>(L.zt64);
    r.C64 = prec == PC_PREC_FP64 ? w.at<double>(L.c) : nullptr;
    r.adj = adj;
    r.st = w.st();
    r.rq = a.rq;
    r.rq_cap = a.rq_cap;
    r.recs = a.recs;
    r.rec_count = a.rec_count;
    r.rec_cap = a.rec_cap;
    r.n = n;
    r.m = m;
    r.mp = L.mp;
    r.W = W;
    r.level = level;
    r.audit = a.force_recheck;
    r.tau = tau;
    PC_HIP(launch_recheck(s, r, auto_grid(ctx)));
    if (e2) PC_HIP(hipEventRecord(e2, s));
    return PC_OK;
}

pc_status read_state(pc_ctx *ctx, const Ws &w) {
    PC_HIP(hipMemcpyAsync(ctx->host_state, w.st(), sizeof(DevState), hipMemcpyDeviceToHost, ctx->stream));
    PC_HIP(hipStreamSynchronize(ctx->stream));
    return PC_OK;
}

void fill_level_stats(pc_run_stats *st, const DevState &d, int level) {
    if (!st || level > PC_MAX_LEVEL) return;
    st->tests[level] = d.tests[level];
    st->removed[level] = d.removed[level];
    st->rechecks[level] = d.rechecks[level];
    st->items[level] = d.items[level];
    st->audit_violations[level] = d.audit_viol[level];
    st->max_degree[level] = d.maxdeg[level];
}

pc_status state_error(const DevState &d) {
    if (d.err) return (pc_status)d.err;
    if (d.overflow) return PC_ERR_UNSUPPORTED;
    if (d.rq_overflow) return PC_ERR_WORKSPACE;
    return PC_OK;
}

}  // namespace

extern "C" {

pc_status pc_default_options(pc_options *opt) {
    if (!opt) return PC_ERR_INVALID_ARG;
    *opt = defaults();
    return PC_OK;
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
    if (hipHostMalloc(reinterpret_cast<void **>(&c->host_state), sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return PC_ERR_HIP;
    }
    std::memset(c->host_state, 0, sizeof(DevState));
    for (auto &e : c->ev) {
        if (hipEventCreate(&e) != hipSuccess) e = nullptr;
    }
    *out = c;
    return PC_OK;
}

void pc_destroy(pc_ctx *ctx) {
    if (!ctx) return;
    for (auto &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    (void)hipHostFree(ctx->host_state);
    delete ctx;
}

size_t pc_workspace_bytes(int64_t n, int64_t m, const pc_options *opt) {
    pc_options o = opt ? *opt : defaults();
    if (n < 1 || m < 1) return 0;
    return Layout::make(n, m, o.precision, rq_cap_of(o)).total;
}

pc_status pc_corr(pc_ctx *ctx, const double *X, int64_t m, int64_t n, double alpha, void *ws,
                  size_t ws_bytes, void *C_out, uint64_t *adj_out) {
    if (!ctx || !X) return PC_ERR_INVALID_ARG;
    if (!(alpha > 0.0 && alpha < 1.0)) return PC_ERR_INVALID_ARG;
    pc_status st = check_shape(n, m);
    if (st != PC_OK) return st;
    Ws w;
    if ((st = check_ws(ctx, n, m, ws, ws_bytes, w)) != PC_OK) return st;
    unsigned long long *adj = w.at<unsigned long long>(w.L.adj);
    if ((st = corr_impl(ctx, X, m, n, alpha, w, adj, nullptr)) != PC_OK) return st;
    const size_t esz = ctx->opt.precision == PC_PREC_FP64 ? sizeof(double) : sizeof(float);
    if (C_out) PC_HIP(hipMemcpyAsync(C_out, w.base + w.L.c, esz * n * n, hipMemcpyDeviceToDevice, ctx->stream));
    if (adj_out)
        PC_HIP(hipMemcpyAsync(adj_out, adj, sizeof(uint64_t) * n * words_per_row(n), hipMemcpyDeviceToDevice,
                              ctx->stream));
    return PC_OK;
}

pc_status pc_sync_status(pc_ctx *ctx, void *ws, size_t ws_bytes) {
    if (!ctx) return PC_ERR_INVALID_ARG;
    PC_HIP(hipStreamSynchronize(ctx->stream));
    if (!ws) return PC_OK;
    if (ws_bytes < sizeof(DevState)) return PC_ERR_WORKSPACE;
    PC_HIP(hipMemcpyAsync(ctx->host_state, ws, sizeof(DevState), hipMemcpyDeviceToHost, ctx->stream));
    PC_HIP(hipStreamSynchronize(ctx->stream));
    return state_error(*ctx->host_state);
}

pc_status pc_level(pc_ctx *ctx, int level, int64_t n, int64_t m, double alpha, uint64_t *adj,
                   const pc_sepset *sep, pc_run_stats *st, void *ws, size_t ws_bytes) {
    if (!ctx || !adj || !sep || !sep->count || (!sep->recs && sep->cap > 0)) return PC_ERR_INVALID_ARG;
    if (level < 1 || level > PC_MAX_LEVEL) return PC_ERR_INVALID_ARG;
    if (!(alpha > 0.0 && alpha < 1.0)) return PC_ERR_INVALID_ARG;
    pc_status s = check_shape(n, m);
    if (s != PC_OK) return s;
    Ws w;
    if ((s = check_ws(ctx, n, m, ws, ws_bytes, w)) != PC_OK) return s;
    const auto t0 = std::chrono::steady_clock::now();
    const bool run_tests = (double)m - level - 3.0 > 0.0;
    PC_HIP(launch_rearm(ctx->stream, w.st()));
    hipEvent_t *ev = ctx->opt.timing ? ctx->ev : nullptr;
    s = level_launch(ctx, level, n, m, alpha, w, reinterpret_cast<unsigned long long *>(adj), sep, run_tests,
                     ev ? ev[0] : nullptr, ev ? ev[1] : nullptr, ev ? ev[2] : nullptr);
    if (s != PC_OK) return s;
    if ((s = read_state(ctx, w)) != PC_OK) return s;
    const DevState &d = *ctx->host_state;
    if ((s = state_error(d)) != PC_OK) return s;
    if (st) {
        fill_level_stats(st, d, level);
        if (ev && run_tests) {
            (void)hipEventElapsedTime(&st->compact_ms[level], ev[0], ev[1]);
            (void)hipEventElapsedTime(&st->level_ms[level], ev[1], ev[2]);
        }
        st->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (!run_tests && !d.done) return PC_WARN_SAMPLE_LIMIT;
    long long cnt = 0;
    PC_HIP(hipMemcpy(&cnt, sep->count, sizeof(cnt), hipMemcpyDeviceToHost));
    if (cnt > sep->cap) return PC_ERR_SEPSET_CAPACITY;
    return PC_OK;
}

pc_status pc_skeleton(pc_ctx *ctx, const double *X, int64_t m, int64_t n, double alpha,
                      int max_level, uint64_t *adj_out, const pc_sepset *sep, pc_run_stats *st,
                      void *ws, size_t ws_bytes) {
    if (!ctx || !X || !adj_out || !sep || !sep->count || (!sep->recs && sep->cap > 0))
        return PC_ERR_INVALID_ARG;
    if (!(alpha > 0.0 && alpha < 1.0)) return PC_ERR_INVALID_ARG;
    pc_status s = check_shape(n, m);
    if (s != PC_OK) return s;
    Ws w;
    if ((s = check_ws(ctx, n, m, ws, ws_bytes, w)) != PC_OK) return s;
    const auto t0 = std::chrono::steady_clock::now();
    if (st) std::memset(st, 0, sizeof(*st));
    unsigned long long *adj = reinterpret_cast<unsigned long long *>(adj_out);
    hipEvent_t *ev = ctx->opt.timing ? ctx->ev : nullptr;
    if (ev) PC_HIP(hipEventRecord(ev[2 * (PC_MAX_LEVEL + 2)], ctx->stream));
    if ((s = corr_impl(ctx, X, m, n, alpha, w, adj, reinterpret_cast<long long *>(sep->count))) != PC_OK)
        return s;
    if (ev) PC_HIP(hipEventRecord(ev[2 * (PC_MAX_LEVEL + 2) + 1], ctx->stream));
    pc_status result = PC_OK;
    int levels_run = 1;
    const int cap = max_level >= 0 ? max_level : PC_MAX_LEVEL + 1;
    for (int level = 1; level <= cap && level <= PC_MAX_LEVEL + 1; ++level) {
        const bool sample_ok = (double)m - level - 3.0 > 0.0;
        const bool level_ok = level <= PC_MAX_LEVEL;
        const bool run_tests = sample_ok && level_ok;
        hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
        if (ev && level <= PC_MAX_LEVEL) {
            e0 = ev[2 * level];
            e1 = ev[2 * level + 1];
            e2 = ev[2 * (level + 1)];
        }
        if ((s = level_launch(ctx, level, n, m, alpha, w, adj, sep, run_tests, e0, e1, e2)) != PC_OK) return s;
        if ((s = read_state(ctx, w)) != PC_OK) return s;
        const DevState &d = *ctx->host_state;
        if ((s = state_error(d)) != PC_OK) return s;
        if (d.done) break;
        if (!sample_ok) { result = PC_WARN_SAMPLE_LIMIT; break; }
        if (!level_ok) { result = PC_WARN_LEVEL_CAP; break; }
        levels_run = level + 1;
        if (st && ev) {
            (void)hipEventElapsedTime(&st->compact_ms[level], e0, e1);
            (void)hipEventElapsedTime(&st->level_ms[level], e1, e2);
        }
    }
    if ((s = read_state(ctx, w)) != PC_OK) return s;
    const DevState &d = *ctx->host_state;
    if ((s = state_error(d)) != PC_OK) return s;
    if (st) {
        for (int l = 0; l <= PC_MAX_LEVEL; ++l) fill_level_stats(st, d, l);
        st->max_degree[0] = 0;
        st->levels_run = levels_run;
        if (ev) (void)hipEventElapsedTime(&st->corr_ms, ev[2 * (PC_MAX_LEVEL + 2)], ev[2 * (PC_MAX_LEVEL + 2) + 1]);
    }
    long long cnt = 0;
    PC_HIP(hipMemcpy(&cnt, sep->count, sizeof(cnt), hipMemcpyDeviceToHost));
    if (st)
        st->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (cnt > sep->cap) return PC_ERR_SEPSET_CAPACITY;
    return result;
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
    switch (l) {
#define PC_CASE(K)                                                        \
    case K: {                                                             \
        int Q[K];                                                         \
        comb_unrank<K>(pool, t, Q, binom);                                \
        for (int c = 0; c < K; ++c) P[c] = Q[c];                          \
        break;                                                            \
    }
        PC_CASE(1) PC_CASE(2) PC_CASE(3) PC_CASE(4) PC_CASE(5) PC_CASE(6) PC_CASE(7)
        PC_CASE(8) PC_CASE(9) PC_CASE(10) PC_CASE(11) PC_CASE(12) PC_CASE(13)
#undef PC_CASE
        default: break;
    }
    for (int c = 0; c < l; ++c) out[c] = (skip >= 0 && P[c] >= skip) ? P[c] + 1 : P[c];
    return PC_OK;
}

double pc_threshold(double alpha, double m, int level) {
    if (!(alpha > 0.0 && alpha < 1.0)) return NAN;
    return tau_of(z_of_alpha(alpha), m, level);
}

size_t pc_abi_size(int which) {
    switch (which) {
        case 0: return sizeof(pc_options);
        case 1: return sizeof(pc_sep_rec);
        case 2: return sizeof(pc_sepset);
        case 3: return sizeof(pc_run_stats);
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
