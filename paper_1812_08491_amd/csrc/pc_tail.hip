// The last levels of PC-stable (Algorithm 1, Sec. 2.4) in one work-group per problem.
//
// Once a level holds few CI tests, its four launches (compaction, planning, tests, re-check) cost
// more than the tests: each launch and each work item is a chain of dependent memory round trips.
// k_tail runs every remaining level of a problem inside one work-group, with work-group barriers
// where the level kernels have kernel boundaries:
//   1. the snapshot G' of the rows that can still be tested (degree >= l + 1: degrees only fall,
//      so the list shrinks level by level), one thread compacting each row;
//   2. the stop rule (maximum degree of G' - 1 >= l, Algorithm 2) and the level cap;
//   3. the CI tests of every conditioning set of those rows, with the shared factor and the FP32
//      test with its error band of the level kernel (SetFactor, Eq. 3-6), the live bit checked
//      before every test, removal by the atomic ticket and one SepSet record per removed edge;
//   4. the FP64 re-check of the tests inside the band (Sec. 4.4), from the problem's share of the
//      re-check queue, a wavefront per test.
// A level whose test count (bounded by sum C(d_i, l) (d_i - l) over the rows) exceeds the tail's
// budget, or that is deeper than kTailMaxLevel (beyond it the factor of a 512-thread work-group
// no longer fits in registers), is left to the level kernels:
// tail_next records it, and tail_done the last level the tail finished, so that the level kernels
// neither run a level twice nor overwrite its statistics.
#include "pc_level.h"

namespace pcg {

constexpr int kTailThreads = 512;
constexpr int kTailWaves = kTailThreads / 64;
constexpr int kTailRows = 1024;   // rows that can still be tested, held in LDS
constexpr int kTailBin = 1024;    // binomials C(a, b), a <= max degree, b <= kTailMaxLevel + 1, in LDS
constexpr int kTailRcWaves = 4;   // wavefronts that run the FP64 re-checks
constexpr int kTailMaxLevel = 8;  // deeper levels go back to the level kernels (register budget)
constexpr int kTailBinCols = kTailMaxLevel + 2;

struct TailSmem {
    int rows[kTailRows];              // rows of G' with degree >= l + 1 (ascending)
    int deg[kTailRows];               // their degrees
    unsigned soff[kTailRows + 1];     // exclusive offsets of their conditioning sets
    unsigned long long bin[kTailBin];
    double G[kTailRcWaves][16 * 16];
    double work[kTailRcWaves][kWorks];
    int v[kTailRcWaves][16];
    long long scan_a[kTailWaves], scan_b[kTailWaves];
    int nrows, nnew, maxdeg, nrq, md0;
    unsigned sets;
    unsigned long long bound;
};

// Statistics of a level: per-thread counts summed per wavefront, added to the problem.
__device__ inline void tail_flush(Prob &P, int l, long long tests, long long removed) {
    const long long t = wave_sum_ll(tests), r = wave_sum_ll(removed);
    if ((threadIdx.x & 63) == 0) {
        if (t) add_ll(&P.tests[l], t);
        if (r) add_ll(&P.removed[l], r);
    }
}

// The CI tests of level L over the staged rows: a conditioning set (its factor built once) per
// `split` threads, which divide its candidates j.
template <typename T, int L>
__device__ void tail_tests(const Batch &b, Prob &P, int pd, TailSmem &sm, RqEntry *rq, long long rq_share,
                           bool bin_lds) {
    const int tid = threadIdx.x;
    const int64_t n = P.n, W = P.W;
    const T *C = static_cast<const T *>(P.C);
    const int nr = sm.nnew;
    const unsigned total = sm.sets;
    const double tau = P.tau[L];
    const float tl = P.t[L], band = P.band[L];
    const TableBinom gbin{b.binom};
    const LdsBinom lbin{(lds_ptr<const unsigned long long>)sm.bin, kTailBinCols};
    int split = 1;
    while (split < 64 && (unsigned long long)split * 2 * total <= kTailThreads) split *= 2;
    const int slice = tid % split, groups = kTailThreads / split;
    long long my_tests = 0, my_removed = 0;
    for (unsigned q = (unsigned)(tid / split); q < total; q += (unsigned)groups) {
        // row of set q: the last staged row whose first set is <= q
        int lo = 0, hi = nr;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (sm.soff[mid] <= q) lo = mid;
            else hi = mid;
        }
        const int row = sm.rows[lo], d = sm.deg[lo];
        int P_[L];
        if (bin_lds) comb_unrank<L>(d, (unsigned long long)(q - sm.soff[lo]), P_, lbin);
        else comb_unrank<L>(d, (unsigned long long)(q - sm.soff[lo]), P_, gbin);
        const int *nb = P.nbr + (int64_t)row * n;
        int sid[L];
#pragma unroll
        for (int c = 0; c < L; ++c) sid[c] = nb[P_[c]];
        auto CS = [&](int p, int r) -> T {
            if (p == r) return (T)1;
            return C[(int64_t)nb[p] * n + nb[r]];
        };
        auto CI = [&](int p) -> T { return C[(int64_t)row * n + nb[p]]; };
        SetFactor<T, L> f;
        f.build(P_, CS, CI);
        unsigned long long *arow = P.adj + (int64_t)row * W;
        constexpr int kB = L <= 3 ? 4 : (L <= 7 ? 2 : 1);
        for (int p0 = slice; p0 < d; p0 += kB * split) {
            // kB candidates at once: ids, then liveness and the values of their tests.
            int jb[kB];
            bool go[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int p = p0 + u * split;
                bool ok = p < d;
#pragma unroll
                for (int c = 0; c < L; ++c) ok &= P_[c] != p;
                go[u] = ok;
                jb[u] = ok ? nb[p] : 0;
            }
            T col[kB][L], cij[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int j = jb[u];
                go[u] = go[u] && ((live_word(arow + (j >> 6)) >> (j & 63)) & 1ull);
                // C[S_r, j] from the rows of the set (C is exactly symmetric): the threads sharing a
                // set read ascending columns of the same rows
#pragma unroll
                for (int r = 0; r < L; ++r) col[u][r] = go[u] ? C[(int64_t)sid[r] * n + j] : (T)0;
                cij[u] = go[u] ? C[(int64_t)row * n + j] : (T)0;
            }
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                if (!go[u]) continue;
                const int j = jb[u];
                ++my_tests;
                const int dec = f.test_vals(col[u], cij[u], tau, tl, band);
                if (dec == 1) {
                    const int elo = row < j ? row : j, ehi = row < j ? j : row;
                    if (take_edge(P.adj, W, elo, ehi)) {
                        ++my_removed;
                        write_record(P, elo, ehi, L, sid);
                    }
                } else if (dec == 2) {
                    const int slot = atomicAdd(&sm.nrq, 1);
                    if (slot < rq_share) {
                        RqEntry *e = rq + slot;
                        e->prob = pd;
                        e->i = row;
                        e->j = j;
                        e->cls = 2;
#pragma unroll
                        for (int c = 0; c < PC_MAX_LEVEL; ++c) e->S[c] = c < L ? (uint16_t)sid[c] : (uint16_t)0xffff;
                    } else {
                        atomicOr(&b.st->rq_overflow_tail, 1);
                    }
                }
            }
        }
    }
    tail_flush(P, L, my_tests, my_removed);
}

template <typename T, int L, int LMAX>
struct TailLevels {
    __device__ static void run(int level, const Batch &b, Prob &P, int pd, TailSmem &sm, RqEntry *rq,
                               long long rq_share, bool bin_lds) {
        if (level == L) tail_tests<T, L>(b, P, pd, sm, rq, rq_share, bin_lds);
        else TailLevels<T, L + 1, LMAX>::run(level, b, P, pd, sm, rq, rq_share, bin_lds);
    }
};
template <typename T, int LMAX>
struct TailLevels<T, LMAX + 1, LMAX> {
    __device__ static void run(int, const Batch &, Prob &, int, TailSmem &, RqEntry *, long long, bool) {}
};

// FP64 re-check of the queued tests [0, count) of level l (wavefronts 0 .. kTailRcWaves - 1).
__device__ void tail_recheck(const Batch &b, Prob &P, int pd, TailSmem &sm, const RqEntry *rq, int count, int l) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (wave >= kTailRcWaves) return;
    const int k = l + 2;
    double *Gw = sm.G[wave];
    int *vw = sm.v[wave];
    RcStats rs;
    for (int e = wave; e < count; e += kTailRcWaves) {
        const RqEntry *qe = rq + e;
        if (lane < 16) vw[lane] = lane == 0 ? qe->i : (lane == 1 ? qe->j : (lane < k ? (int)qe->S[lane - 2] : -1));
        const int cls = qe->cls;
        wave_sync();
        if (b.prec != PC_PREC_FP64 && k <= 4) {
            double sp[6];
            gram_small_part(P, vw, k, lane, 0, 128, sp);
#pragma unroll
            for (int q = 0; q < 6; ++q) sp[q] = wave_sum64(sp[q]);
            if (lane == 0) gram_small_store(sp, k, Gw);
        } else if (b.prec != PC_PREC_FP64) {
            const doublex4 acc = gram_part<1>(P, vw[lane & 15], lane, 0, 64);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int rr = (lane >> 4) + 4 * t, cc = lane & 15;
                Gw[rr * 16 + cc] = rr == cc ? 1.0 : acc[t];
            }
        } else {
            for (int q = lane; q < k * k; q += 64) {
                const int rr = q / k, cc = q % k;
                Gw[rr * 16 + cc] = rr == cc ? 1.0 : static_cast<const double *>(P.C)[(int64_t)vw[rr] * P.n + vw[cc]];
            }
        }
        wave_sync();
        const int res = decide_wave<16>(Gw, 16, l, P.tau[l], sm.work[wave], kMMs, lane);
        if (lane == 0) {
            rs.at(b, l, pd);
            settle_recheck(b, P, l, res, vw[0], vw[1], cls, vw + 2, rs);
        }
        wave_sync();
    }
    if (lane == 0) rs.flush(b, l);
}

template <typename T>
__global__ __launch_bounds__(kTailThreads) void k_tail(Batch b, int level0, long long cap_tests) {
    __shared__ TailSmem sm;
    const int tid = threadIdx.x, lane = tid & 63;
    if (b.st->done) return;
    const int pd = blockIdx.x;
    Prob &P = b.probs[pd];
    if (P.err) return;
    const int64_t n = P.n, W = P.W;
    const TableBinom gbin{b.binom};
    // This problem's share of the re-check queue (the level kernels' queue is idle meanwhile).
    const long long rq_share = b.rq_cap / b.count;
    RqEntry *rq = b.rq + (long long)pd * rq_share;

    // Rows that can still be tested at level0: degree >= level0 + 1 in the last snapshot.
    if (tid == 0) {
        sm.nrows = 0;
        sm.md0 = 0;
    }
    __syncthreads();
    int dmax = 0;
    for (int r0 = 0; r0 < n; r0 += kTailThreads) {
        const int r = r0 + tid;
        const int dr = r < n ? P.deg[r] : 0;
        const bool f = dr >= level0 + 1;
        dmax = f && dr > dmax ? dr : dmax;
        long long tot = 0;
        const long long pre = block_exclusive_scan<kTailThreads>(f ? 1 : 0, sm.scan_a, tot);
        const int base = sm.nrows;
        if (f && base + pre < kTailRows) sm.rows[base + pre] = r;
        __syncthreads();
        if (tid == 0) sm.nrows = base + (int)tot;
        __syncthreads();
    }
    for (int o = 32; o >= 1; o >>= 1) {
        const int om = __shfl_xor(dmax, o, 64);
        dmax = om > dmax ? om : dmax;
    }
    if (lane == 0) atomicMax(&sm.md0, dmax);
    __syncthreads();
    // Binomials of every unranking and count of the tail: degrees never exceed md0 again.
    const int md0 = sm.md0;
    const bool bin_lds = (md0 + 1) * kTailBinCols <= kTailBin;
    if (bin_lds)
        for (int e = tid; e < (md0 + 1) * kTailBinCols; e += kTailThreads)
            sm.bin[e] = gbin(e / kTailBinCols, e % kTailBinCols);
    __syncthreads();
    const LdsBinom lbin{(lds_ptr<const unsigned long long>)sm.bin, kTailBinCols};
    auto binom = [&](int a, int k) -> unsigned long long { return bin_lds ? lbin(a, k) : gbin(a, k); };
    int level = level0, stop = 0;   // stop: 1 finished, 2 left to the level kernels
    if (sm.nrows > kTailRows) stop = 2;
    while (!stop) {
        const int nr = sm.nrows;
        if (tid == 0) {
            sm.maxdeg = 0;
            sm.nrq = 0;
            sm.nnew = 0;
            sm.sets = 0;
            sm.bound = 0;
        }
        __syncthreads();
        // 1. G' of the staged rows (live bits read past the vector caches: removals are atomics).
        int mymax = 0;
        unsigned long long mybound = 0;
        for (int q = tid; q < nr; q += kTailThreads) {
            const int r = sm.rows[q];
            unsigned long long *arow = P.adj + (int64_t)r * W;
            int *out = P.nbr + (int64_t)r * n;
            int cnt = 0;
            for (int64_t w0 = 0; w0 < W; w0 += 16) {
                unsigned long long wd[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) wd[u] = w0 + u < W ? live_word(arow + w0 + u) : 0ull;
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int64_t w = w0 + u;
                    unsigned long long x = wd[u];
                    if (w == (r >> 6)) x &= ~(1ull << (r & 63));
                    if (w == W - 1 && (n & 63)) x &= (1ull << (n & 63)) - 1ull;
                    while (x) {
                        out[cnt++] = (int)(w * 64 + (__ffsll((long long)x) - 1));
                        x &= x - 1;
                    }
                }
            }
            P.deg[r] = cnt;
            sm.deg[q] = cnt;
            mymax = cnt > mymax ? cnt : mymax;
            if (cnt >= level + 1) {
                // tests of the row: C(d, l) sets of d - l candidates (saturating at 2^50 per thread)
                constexpr unsigned long long kSatB = 1ull << 50;
                const unsigned long long c = binom(cnt, level);
                const unsigned long long t = c < (1ull << 30) ? c * (unsigned long long)(cnt - level) : kSatB;
                mybound = mybound + t < kSatB ? mybound + t : kSatB;
            }
        }
        for (int o = 32; o >= 1; o >>= 1) {
            const int om = __shfl_xor(mymax, o, 64);
            mymax = om > mymax ? om : mymax;
        }
        const unsigned long long wb = wave_sum_ll((long long)mybound);
        if (lane == 0) {
            atomicMax(&sm.maxdeg, mymax);
            atomicAdd(&sm.bound, wb);
        }
        __syncthreads();
        const int md = sm.maxdeg;
        // 2. Stop rule and level cap (the statistics of a level record its G' maximum degree).
        if (md < level + 1 || !level_enabled(P, level)) {
            if (tid == 0) P.maxdeg[level] = md;
            stop = 1;
            break;
        }
        if (level > kTailMaxLevel || sm.bound > (unsigned long long)cap_tests) {
            stop = 2;
            break;
        }
        if (tid == 0) P.maxdeg[level] = md;
        // The rows with degree >= level + 1, with the offsets of their conditioning sets.
        for (int q0 = 0; q0 < nr; q0 += kTailThreads) {
            const int q = q0 + tid;
            int r = 0, dq = 0;
            bool f = false;
            unsigned long long ns = 0;
            if (q < nr) {
                r = sm.rows[q];
                dq = sm.deg[q];
                f = dq >= level + 1;
                ns = f ? binom(dq, level) : 0;
            }
            long long tot = 0, stot = 0;
            const long long pre = block_exclusive_scan<kTailThreads>(f ? 1 : 0, sm.scan_a, tot);
            const long long spre = block_exclusive_scan<kTailThreads>((long long)ns, sm.scan_b, stot);
            const int base = sm.nnew;
            const unsigned sbase = sm.sets;
            __syncthreads();
            if (f) {
                sm.rows[base + pre] = r;
                sm.deg[base + pre] = dq;
                sm.soff[base + pre] = sbase + (unsigned)spre;
            }
            __syncthreads();
            if (tid == 0) {
                sm.nnew = base + (int)tot;
                sm.sets = sbase + (unsigned)stot;
            }
            __syncthreads();
        }
        if (tid == 0) {
            sm.soff[sm.nnew] = sm.sets;
            P.items[level] = sm.sets;
        }
        __syncthreads();
        // 3. The tests of the level.
        TailLevels<T, 1, kTailMaxLevel>::run(level, b, P, pd, sm, rq, rq_share, bin_lds);
        __syncthreads();
        // 4. FP64 re-checks of the tests inside the band.
        const int nrq = sm.nrq < rq_share ? sm.nrq : (int)rq_share;
        if (nrq > 0) tail_recheck(b, P, pd, sm, rq, nrq, level);
        __syncthreads();
        if (tid == 0) {
            P.tail_done = level;
            sm.nrows = sm.nnew;
        }
        __syncthreads();
        ++level;
    }
    if (tid == 0) {
        if (stop == 1) {
            P.tail_done = level;
            P.tail_next = 0;
        } else {
            P.tail_done = level - 1;
            P.tail_next = level;
        }
    }
}

hipError_t launch_tail(hipStream_t s, const Batch &b, int level, long long cap_tests) {
    if (level < 1) return hipErrorInvalidValue;
    if (b.prec == PC_PREC_FP64)
        hipLaunchKernelGGL(k_tail<double>, dim3((unsigned)b.count), dim3(kTailThreads), 0, s, b, level, cap_tests);
    else
        hipLaunchKernelGGL(k_tail<float>, dim3((unsigned)b.count), dim3(kTailThreads), 0, s, b, level, cap_tests);
    return hipGetLastError();
}

}  // namespace pcg
