// Compaction, planning and the per-level dispatch of PC-stable's levels l >= 1 (Algorithm 1,
// Sec. 2.4); the level kernels themselves are described in pc_level.h.
#include "pc_level.h"

namespace pcg {

// ---------------------------------------------------------------------------------------------
// Compaction and planning
// ---------------------------------------------------------------------------------------------
constexpr unsigned long long kMaxSetsPerRow = 1ull << 40;

// Work items of a row of degree `count` at `level` within the launch's rank window (0 when the
// row has fewer than level + 1 neighbours or the level is disabled for its problem).
__device__ inline long long row_items(const Batch &b, const Prob &P, int count, int level, int R) {
    if (count < level + 1 || !level_enabled(P, level)) return 0;
    const unsigned long long nS = b.binom[(int64_t)count * kBinomCols + level];
    if (nS > kMaxSetsPerRow) {
        atomicOr(&b.st->overflow, 1);
        return 0;
    }
    unsigned long long lo, hi;
    rank_window(b, nS, lo, hi);
    const unsigned long long r = (unsigned long long)item_sets(count, level, R, b.lane_tests);
    return (long long)((hi - lo + r - 1) / r);
}

__global__ __launch_bounds__(256) void k_compact(Batch b, int level, int R) {
    if (b.st->done) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long grow = (long long)blockIdx.x * 4 + wave;
    if (grow >= b.total_rows) return;
    const int d = find_base(b.row_base, b.count, grow);
    Prob &P = b.probs[d];
    const int64_t n = P.n, W = P.W, i = grow - b.row_base[d];
    const unsigned long long *row = P.adj + i * W;
    int *out = P.nbr + i * n;
    int count = 0;
    for (int64_t w0 = 0; w0 < W; w0 += 64) {
        const int64_t w = w0 + lane;
        unsigned long long word = w < W ? row[w] : 0ull;
        // A caller-supplied G may carry stray bits: drop the diagonal and columns >= n.
        if (w == (i >> 6)) word &= ~(1ull << (i & 63));
        if (w == W - 1 && (n & 63)) word &= (1ull << (n & 63)) - 1ull;
        const int pc = __popcll(word);
        int incl = pc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        const int tot = __shfl(incl, 63, 64);
        int pos = count + incl - pc;
        while (word) {
            const int bit = __ffsll((long long)word) - 1;
            out[pos++] = (int)(w * 64 + bit);
            word &= word - 1;
        }
        count += tot;
    }
    if (lane == 0) {
        P.deg[i] = count;
        b.nitems[grow] = row_items(b, P, count, level, R);
        b.rowdeg[grow] = count;
        b.rowdeg[b.total_rows + grow] = d;
    }
}

// Per row of G': work items of a launch's rank window, from the degree the compaction stored.
__global__ __launch_bounds__(256) void k_window(Batch b, int level, int R) {
    if (b.st->done) return;
    const long long grow = (long long)blockIdx.x * 256 + threadIdx.x;
    if (grow >= b.total_rows) return;
    const int d = find_base(b.row_base, b.count, grow);
    const Prob &P = b.probs[d];
    b.nitems[grow] = row_items(b, P, P.deg[grow - b.row_base[d]], level, R);
}

hipError_t launch_compact(hipStream_t s, const Batch &b, int level, int ranks_per_item) {
    const dim3 grid((unsigned)((b.total_rows + 3) / 4));
    hipLaunchKernelGGL(k_compact, grid, dim3(256), 0, s, b, level, ranks_per_item);
    return hipGetLastError();
}

// Order in which the queue hands out a level's items. Items are numbered row by row, so when rows
// have many items each (long rows of a dense G'), handing them out in that order would set every
// resident work-group on the same few rows at once: all of them would test those rows against the
// same still-live candidates, and race to remove the same edges. With several items per row on
// average, pop g takes item (g * s) mod total instead, s about the number of rows and coprime to
// the total (a permutation): consecutive pops fall on different rows, and a row's items are spread
// over the whole launch, so its later items see the removals of its earlier ones.
__device__ inline unsigned long long item_stride(long long total, long long rows) {
    if (rows < 2 || total < 4 * rows) return 1ull;
    unsigned long long s = (unsigned long long)rows;
    for (;;) {
        unsigned long long a = s, c = (unsigned long long)total;
        while (c) {
            const unsigned long long t = a % c;
            a = c;
            c = t;
        }
        if (a == 1ull) return s;
        ++s;
    }
}

constexpr int kPlanThreads = 1024;
constexpr int kPlanPer = 4;                           // rows per thread in a tile
constexpr int kPlanTile = kPlanThreads * kPlanPer;    // rows per tile
constexpr int kPlanLdsProbs = 4096;     // problems whose max degree is reduced in LDS

// One work-group plans the level for the whole batch. The per-row values are read a tile of
// kPlanTile rows at a time with coalesced loads into LDS (a wavefront reads consecutive rows), and
// each thread then works on kPlanPer consecutive rows of the tile from LDS: with one thread per
// contiguous chunk of rows in global memory instead, every load instruction of a wavefront would
// touch 64 different cache lines of the one CU that runs the plan. The loads of the next tile are
// in flight while the current one is scanned.
__global__ __launch_bounds__(kPlanThreads) void k_plan(Batch b, int level, int window) {
    __shared__ long long part[kPlanThreads / 64];
    __shared__ long long t_items[kPlanTile];   // work items, then their offsets
    __shared__ int t_deg[kPlanTile], t_prob[kPlanTile];
    __shared__ int s_maxdeg[kPlanLdsProbs];
    DevState *st = b.st;
    if (st->done) return;
    const int tid = threadIdx.x;
    const long long N = b.total_rows;
    // Max degree of G' per problem (what the stop rule of Algorithm 1 looks at): segment maxima of
    // a thread's rows meet in LDS (one slot per problem) when the batch is small enough, so no
    // global address sees more than one write per problem.
    const bool in_lds = b.count <= kPlanLdsProbs;
    const bool degrees = !window;
    if (degrees && in_lds)
        for (int d = tid; d < b.count; d += kPlanThreads) s_maxdeg[d] = 0;
    auto flush = [&](int d, int best) {
        if (d < 0 || best <= 0) return;
        if (in_lds) atomicMax(&s_maxdeg[d], best);
        else if (level > b.probs[d].tail_done) atomicMax(&b.probs[d].maxdeg[level], best);
    };
    long long v[kPlanPer];
    int dg[kPlanPer], pr[kPlanPer];
    auto fetch = [&](long long t0) {
#pragma unroll
        for (int u = 0; u < kPlanPer; ++u) {
            const long long r = t0 + (long long)u * kPlanThreads + tid;
            v[u] = r < N ? b.nitems[r] : 0;
            dg[u] = degrees && r < N ? b.rowdeg[r] : 0;
            pr[u] = degrees && r < N ? b.rowdeg[N + r] : -1;
        }
    };
    fetch(0);
    long long carry = 0;
    for (long long t0 = 0; t0 < N; t0 += kPlanTile) {
#pragma unroll
        for (int u = 0; u < kPlanPer; ++u) {
            t_items[u * kPlanThreads + tid] = v[u];
            t_deg[u * kPlanThreads + tid] = dg[u];
            t_prob[u * kPlanThreads + tid] = pr[u];
        }
        if (t0 + kPlanTile < N) fetch(t0 + kPlanTile);
        __syncthreads();
        long long a[kPlanPer], s = 0;
#pragma unroll
        for (int u = 0; u < kPlanPer; ++u) {
            a[u] = t_items[kPlanPer * tid + u];
            s += a[u];
        }
        if (degrees) {
            int cur = -1, best = 0;
#pragma unroll
            for (int u = 0; u < kPlanPer; ++u) {
                const int p = t_prob[kPlanPer * tid + u], x = t_deg[kPlanPer * tid + u];
                if (p != cur) {
                    flush(cur, best);
                    cur = p;
                    best = 0;
                }
                best = x > best ? x : best;
            }
            flush(cur, best);
        }
        long long tot = 0;
        long long run = carry + block_exclusive_scan<kPlanThreads>(s, part, tot);
#pragma unroll
        for (int u = 0; u < kPlanPer; ++u) {
            t_items[kPlanPer * tid + u] = run;
            run += a[u];
        }
        carry += tot;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPlanPer; ++u) {
            const long long r = t0 + (long long)u * kPlanThreads + tid;
            if (r < N) b.item_off[r] = t_items[u * kPlanThreads + tid];
        }
        __syncthreads();   // the tiles and the scan's LDS are refilled next
    }
    const long long total = carry;
    if (tid == 0) {
        b.item_off[N] = total;
        st->total_items = (unsigned long long)total;
        st->next_item = 0ull;
        st->item_stride = item_stride(total, N);
        if (!window && total == 0) st->done = 1;
    }
    if (window) return;   // a window of a planned level: its statistics and stop flag stand
    if (tid < kRqSlices) st->rq_slice[tid] = 0ull;   // a new level's re-check queue
    __syncthreads();
    // Levels the tail kernel already ran keep the statistics it recorded.
    for (int d = tid; d < b.count; d += kPlanThreads)
        if (level > b.probs[d].tail_done) {
            b.probs[d].items[level] = b.item_off[b.row_base[d + 1]] - b.item_off[b.row_base[d]];
            if (in_lds) b.probs[d].maxdeg[level] = s_maxdeg[d];
        }
}

hipError_t launch_plan(hipStream_t s, const Batch &b, int level) {
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(kPlanThreads), 0, s, b, level, 0);
    return hipGetLastError();
}

hipError_t launch_window(hipStream_t s, const Batch &b, int level, int ranks_per_item) {
    hipLaunchKernelGGL(k_window, dim3((unsigned)((b.total_rows + 255) / 256)), dim3(256), 0, s, b, level,
                       ranks_per_item);
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(kPlanThreads), 0, s, b, level, 1);
    return hipGetLastError();
}

size_t level_lds_fixed(int prec) {
    return prec == PC_PREC_FP64 ? lds_fixed_bytes<double>() : lds_fixed_bytes<float>();
}

int level_blocks_per_cu(int prec, int level, int lds_bytes) {
    if (level < 1 || level > PC_MAX_LEVEL) return 0;
    if (level > kFastLevels) return occupancy_level_deep(prec, level);
    return prec == PC_PREC_FP64 ? occupancy_level_fast_f64(level, lds_bytes) : occupancy_level_fast_f32(level, lds_bytes);
}

hipError_t launch_level(hipStream_t s, const Batch &b, int level, int R, int lds_bytes, int grid) {
    if (level < 1 || level > PC_MAX_LEVEL) return hipErrorInvalidValue;
    if (level > kFastLevels) return launch_level_deep(s, b, level, R, lds_bytes, grid);
    if (b.prec == PC_PREC_FP64) return launch_level_fast_f64(s, b, level, R, lds_bytes, grid);
    return launch_level_fast_f32(s, b, level, R, lds_bytes, grid);
}

}  // namespace pcg
