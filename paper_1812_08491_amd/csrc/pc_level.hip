// Levels l >= 1 of PC-stable (Algorithm 1, Sec. 2.4) on gfx950, for a batch of problems.
//
// k_compact: the snapshot G' := G as compacted neighbour lists (the A'_G of Sec. 3.3 / Fig. 2):
//   one wavefront per row turns the row's bit words into ascending neighbour ids with popcount and
//   a wave prefix sum, and counts the row's work items (C(d_i, l) conditioning sets, cut into
//   items of a fixed number of ranks; none when d_i < l + 1, Sec. 4.1).
// k_plan: one work-group scans the per-row item counts into the level's work queue. A level with
//   no work in any problem sets the device stop flag: the max-degree test of Algorithm 2, kept on
//   the device so that no host round trip is needed between levels.
// k_level<T, L>: the CI tests of level L. A work item is a row i with a range of ranks of its
//   l-subsets S of adj(i, G') (the set-sharing view of cuPC-S, Sec. 3.4): for each S the
//   Cholesky factor of M2 = C[S,S] (Eq. 3) is formed once and serves every j in adj(i,G') \ S, so
//   the per-j work is one triangular solve. The row's neighbour list, C[i, N_i], its live bits and
//   (when it fits) the block C[N_i, N_i] are staged in LDS once per item. Items come from a
//   device-side queue that a fixed grid of work-groups drains (persistent kernel), absorbing the
//   very uneven per-row subset counts.
//   Every test first checks that edge (i,j) is still in G (early termination, Sec. 4.1). The first
//   independent test clears the edge with an atomic AND on the bit (min, max); only the thread
//   whose AND cleared it writes the SepSet record, so each removed edge has exactly one record.
//   FP32 tests whose |rho| lies within an error band of tanh(tau_l) (and FP64 tests whose M2 is
//   rank deficient) go to a re-check queue.
// k_recheck: one wavefront per queued test re-evaluates it in FP64 (the block of C recomputed as
//   dot products of the FP64 standardized columns, or read from the FP64 C), with a
//   pseudo-inverse when M2 is rank deficient, and removes the edge if that decides independence.
#include "pc_citest.h"
#include "pc_comb.h"
#include "pc_dev.h"

namespace pcg {

__device__ inline double wave_sum64(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline long long wave_sum_ll(long long v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Adds a work-group's test and removal counts of level L to its problem and clears them.
template <int L>
__device__ inline void flush_stats(Prob &P, long long &tests, long long &removed) {
    if (tests) add_ll(&P.tests[L], tests);
    if (removed) add_ll(&P.removed[L], removed);
    tests = 0;
    removed = 0;
}

// Whether level l runs for problem P (the level cap, Eq. 6 needing m - l - 3 > 0).
__device__ inline bool level_enabled(const Prob &P, int l) {
    return l <= P.max_level && l <= PC_MAX_LEVEL && P.tau[l] == P.tau[l];
}

// ---------------------------------------------------------------------------------------------
// Compaction and planning
// ---------------------------------------------------------------------------------------------
constexpr unsigned long long kMaxSetsPerRow = 1ull << 40;

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
        long long items = 0;
        if (count >= level + 1 && level_enabled(P, level)) {
            const unsigned long long nS = b.binom[(int64_t)count * kBinomCols + level];
            if (nS > kMaxSetsPerRow) {
                atomicOr(&b.st->overflow, 1);
            } else {
                items = (long long)((nS + (unsigned long long)R - 1) / (unsigned long long)R);
            }
        }
        b.nitems[grow] = items;
    }
}

hipError_t launch_compact(hipStream_t s, const Batch &b, int level, int ranks_per_item) {
    const dim3 grid((unsigned)((b.total_rows + 3) / 4));
    hipLaunchKernelGGL(k_compact, grid, dim3(256), 0, s, b, level, ranks_per_item);
    return hipGetLastError();
}

constexpr int kPlanThreads = 1024;
constexpr int kPlanLdsProbs = 4096;     // problems whose max degree is reduced in LDS

__global__ __launch_bounds__(kPlanThreads) void k_plan(Batch b, int level) {
    __shared__ long long part[kPlanThreads / 64];
    DevState *st = b.st;
    if (st->done) return;
    const int tid = threadIdx.x;
    const long long N = b.total_rows;
    const long long chunk = (N + kPlanThreads - 1) / kPlanThreads;
    const long long lo = tid * chunk, hi = lo + chunk < N ? lo + chunk : N;
    long long s = 0;
    for (long long k = lo; k < hi; ++k) s += b.nitems[k];
    long long total = 0;
    long long run = block_exclusive_scan<kPlanThreads>(s, part, total);
    for (long long k = lo; k < hi; ++k) {
        b.item_off[k] = run;
        run += b.nitems[k];
    }
    if (tid == 0) {
        b.item_off[N] = total;
        st->total_items = (unsigned long long)total;
        st->next_item = 0ull;
        st->rq_count = 0ull;
        if (total == 0) st->done = 1;
    }
    __syncthreads();
    for (int d = tid; d < b.count; d += kPlanThreads)
        b.probs[d].items[level] = b.item_off[b.row_base[d + 1]] - b.item_off[b.row_base[d]];
    // Max degree of G' per problem (what the stop rule of Algorithm 1 looks at). Each thread scans
    // its chunk of rows segment by segment; segment maxima meet in LDS (one slot per problem) when
    // the batch is small enough, so no global address sees more than one write per problem.
    const bool in_lds = b.count <= kPlanLdsProbs;
    __shared__ int s_maxdeg[kPlanLdsProbs];
    if (in_lds)
        for (int d = tid; d < b.count; d += kPlanThreads) s_maxdeg[d] = 0;
    __syncthreads();
    if (lo < hi) {
        int d = find_base(b.row_base, b.count, lo);
        int best = 0;
        for (long long k = lo; k < hi; ++k) {
            while (k >= b.row_base[d + 1]) {
                if (best > 0) {
                    if (in_lds) atomicMax(&s_maxdeg[d], best);
                    else atomicMax(&b.probs[d].maxdeg[level], best);
                }
                best = 0;
                ++d;
            }
            const int dg = b.probs[d].deg[k - b.row_base[d]];
            best = dg > best ? dg : best;
        }
        if (best > 0) {
            if (in_lds) atomicMax(&s_maxdeg[d], best);
            else atomicMax(&b.probs[d].maxdeg[level], best);
        }
    }
    if (in_lds) {
        __syncthreads();
        for (int d = tid; d < b.count; d += kPlanThreads) b.probs[d].maxdeg[level] = s_maxdeg[d];
    }
}

hipError_t launch_plan(hipStream_t s, const Batch &b, int level) {
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(kPlanThreads), 0, s, b, level);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// FP64 decision from a Gram block (used by the re-check)
// ---------------------------------------------------------------------------------------------

// Per-wave FP64 scratch of the re-check path, kept in LDS (runtime-sized small matrices).
constexpr int kMM = PC_MAX_LEVEL * PC_MAX_LEVEL;
constexpr int kWork = 4 * kMM + 2 * PC_MAX_LEVEL;   // Lm, a, v, P, y, w (levels up to PC_MAX_LEVEL)
constexpr int kMMs = 14 * 14;                       // the same for levels up to 14 (16 variables)
constexpr int kWorks = 4 * kMMs + 2 * 14;

// Moore-Penrose inverse of the symmetric k x k block A (row stride lda) by cyclic Jacobi
// rotations (Sec. 4.4 asks for a pseudo-inverse of M2; the eigen route gives the same unique
// matrix as the paper's full-rank Cholesky route). Eigenvalues <= k * eps * lambda_max count as
// zero. a, v, P: k x k scratch with stride k.
__device__ void pinv_jacobi(const double *A, int lda, int k, double *a, double *v, double *P) {
    for (int r = 0; r < k; ++r)
        for (int c = 0; c < k; ++c) {
            a[r * k + c] = A[r * lda + c];
            v[r * k + c] = r == c ? 1.0 : 0.0;
        }
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, all = 0.0;
        for (int r = 0; r < k; ++r)
            for (int c = 0; c < k; ++c) {
                const double e = a[r * k + c] * a[r * k + c];
                all += e;
                if (r != c) off += e;
            }
        if (off == 0.0 || off <= 1e-32 * all) break;
        for (int p = 0; p < k - 1; ++p)
            for (int q = p + 1; q < k; ++q) {
                const double apq = a[p * k + q];
                if (apq == 0.0) continue;
                const double th = (a[q * k + q] - a[p * k + p]) / (2.0 * apq);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int r = 0; r < k; ++r) {
                    const double x = a[r * k + p], y = a[r * k + q];
                    a[r * k + p] = cs * x - sn * y;
                    a[r * k + q] = sn * x + cs * y;
                }
                for (int r = 0; r < k; ++r) {
                    const double x = a[p * k + r], y = a[q * k + r];
                    a[p * k + r] = cs * x - sn * y;
                    a[q * k + r] = sn * x + cs * y;
                }
                for (int r = 0; r < k; ++r) {
                    const double x = v[r * k + p], y = v[r * k + q];
                    v[r * k + p] = cs * x - sn * y;
                    v[r * k + q] = sn * x + cs * y;
                }
            }
    }
    double lmax = 0.0;
    for (int r = 0; r < k; ++r) lmax = fmax(lmax, fabs(a[r * k + r]));
    const double cut = (double)k * 2.220446049250313e-16 * lmax;
    for (int r = 0; r < k; ++r)
        for (int c = 0; c < k; ++c) {
            double s = 0.0;
            for (int e = 0; e < k; ++e)
                if (a[e * k + e] > cut) s += v[r * k + e] * v[c * k + e] / a[e * k + e];
            P[r * k + c] = s;
        }
}

// G: (l+2) x (l+2) correlation block over (i, j, S...), row stride ld. Returns 1 iff the Fisher z
// of rho(i,j|S) (Eq. 3-5) is <= tau. Rules: M2 through its Cholesky factor unless a pivot is
// <= 1e-12 * max diag(M2), then through its pseudo-inverse; H11 <= 0 or H22 <= 0 gives rho = 0.
// work: 4 mm + 2 l doubles of scratch, mm >= l * l.
__device__ int decide_gram64(const double *G, int ld, int l, double tau, double *work, int mm) {
    double h11 = 1.0, h22 = 1.0, h12 = G[1];
    if (l > 0) {
        double *Lm = work, *a = work + mm, *v = work + 2 * mm, *P = work + 3 * mm;
        double *y = work + 4 * mm, *w = y + l;
        const double *M2 = G + 2 * ld + 2;
        double maxdiag = 0.0;
        for (int r = 0; r < l; ++r) maxdiag = fmax(maxdiag, M2[r * ld + r]);
        bool ok = true;
        for (int r = 0; r < l && ok; ++r)
            for (int c = 0; c <= r; ++c) {
                double s = M2[r * ld + c];
                for (int e = 0; e < c; ++e) s -= Lm[r * l + e] * Lm[c * l + e];
                if (r == c) {
                    if (!(s > 1e-12 * maxdiag)) { ok = false; break; }
                    Lm[r * l + r] = sqrt(s);
                } else {
                    Lm[r * l + c] = s / Lm[c * l + c];
                }
            }
        if (ok) {
            double yy = 0.0, ww = 0.0, yw = 0.0;
            for (int r = 0; r < l; ++r) {
                double sy = G[2 + r], sw = G[ld + 2 + r];
                for (int e = 0; e < r; ++e) { sy -= Lm[r * l + e] * y[e]; sw -= Lm[r * l + e] * w[e]; }
                y[r] = sy / Lm[r * l + r];
                w[r] = sw / Lm[r * l + r];
                yy += y[r] * y[r];
                ww += w[r] * w[r];
                yw += y[r] * w[r];
            }
            h11 = 1.0 - yy;
            h22 = 1.0 - ww;
            h12 = G[1] - yw;
        } else {
            pinv_jacobi(M2, ld, l, a, v, P);
            double q11 = 0.0, q22 = 0.0, q12 = 0.0;
            for (int r = 0; r < l; ++r)
                for (int c = 0; c < l; ++c) {
                    q11 += G[2 + r] * P[r * l + c] * G[2 + c];
                    q22 += G[ld + 2 + r] * P[r * l + c] * G[ld + 2 + c];
                    q12 += G[2 + r] * P[r * l + c] * G[ld + 2 + c];
                }
            h11 = 1.0 - q11;
            h22 = 1.0 - q22;
            h12 = G[1] - q12;
        }
    }
    const double rho = (h11 > 0.0 && h22 > 0.0) ? h12 / sqrt(h11 * h22) : 0.0;
    return fisher_z64(rho) <= tau ? 1 : 0;
}

// ---------------------------------------------------------------------------------------------
// Level kernel
// ---------------------------------------------------------------------------------------------
constexpr int kStageCap = kLevelThreads;   // removals staged per item (one settling thread each)
constexpr int kDcap = 1024;   // neighbour lists up to this degree are staged in LDS
constexpr int kWcap = 256;    // live-bit words of a row staged in LDS (n <= 16384)

struct TableBinom {
    const unsigned long long *t;
    __device__ unsigned long long operator()(int a, int b) const {
        if (b < 0 || a < b) return 0ull;
        return t[(int64_t)a * kBinomCols + b];
    }
};

template <typename T>
__host__ __device__ constexpr size_t lds_fixed_bytes() {
    return (sizeof(int) * kDcap + 15) / 16 * 16 + (sizeof(T) * kDcap + 15) / 16 * 16 +
           sizeof(unsigned long long) * kWcap;
}

template <typename T, int L>
__global__ __launch_bounds__(kLevelThreads) void k_level(Batch b, int R, int lds_bytes) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ long long s_grow, s_r0;
    __shared__ int s_mode;  // bit 0: nb/ci in LDS, bit 1: C[N_i,N_i] in LDS, bit 2: live bits in LDS
    __shared__ long long s_tests, s_removed;
    // Removals found while testing are staged here and settled at the end of the item, so a
    // wavefront never waits on a device-scope atomic inside the test loop.
    __shared__ int s_nstage, s_nwin;
    __shared__ int s_stage_j[kStageCap];
    __shared__ unsigned long long s_stage_t[kStageCap];
    __shared__ unsigned long long s_rec_base;

    DevState *st = b.st;
    if (st->done) return;
    const unsigned long long total = st->total_items;
    const int tid = threadIdx.x;
    int *lds_nb = reinterpret_cast<int *>(smem);
    T *lds_ci = reinterpret_cast<T *>(smem + (sizeof(int) * kDcap + 15) / 16 * 16);
    unsigned long long *lds_live = reinterpret_cast<unsigned long long *>(
        smem + (sizeof(int) * kDcap + 15) / 16 * 16 + (sizeof(T) * kDcap + 15) / 16 * 16);
    T *lds_blk = reinterpret_cast<T *>(smem + lds_fixed_bytes<T>());
    const long long blk_cap = ((long long)lds_bytes - (long long)lds_fixed_bytes<T>()) / (long long)sizeof(T);
    const TableBinom binom{b.binom};

    if (tid == 0) { s_tests = 0; s_removed = 0; s_nstage = 0; s_nwin = 0; }
    long long staged = -1, last_row = 0;
    int d = 0, stats_pd = -1;
    long long my_tests = 0, my_removed = 0;
    bool first = true;

    for (;;) {
        __syncthreads();
        if (tid < 64) {
            // Wave 0 takes the next item and finds its row: the largest r with item_off[r] <= g,
            // by 64-way probing (each round narrows the range 64-fold with one load per lane).
            // The first item of a work-group is its own index; later ones come from the queue.
            unsigned long long g = blockIdx.x;
            if (!first && tid == 0) g = gridDim.x + atomicAdd(&st->next_item, 1ull);
            g = __shfl(g, 0, 64);
            if (g >= total) {
                if (tid == 0) s_grow = -1;
            } else {
                long long lo = last_row, hi = b.total_rows;
                while (hi - lo > 1) {
                    const long long step = (hi - lo + 63) / 64;
                    const long long idx = lo + (long long)tid * step;
                    const bool ok = idx < hi && (unsigned long long)b.item_off[idx] <= g;
                    const unsigned long long mask = __ballot(ok);
                    const int top = 63 - __clzll((long long)mask);  // lane 0 always qualifies
                    lo = lo + (long long)top * step;
                    hi = lo + step < hi ? lo + step : hi;
                }
                if (tid == 0) {
                    s_grow = lo;
                    s_r0 = (long long)(g - (unsigned long long)b.item_off[lo]) * R;
                }
            }
        }
        __syncthreads();
        first = false;
        const long long grow = s_grow;
        if (grow < 0) break;
        last_row = grow;
        const int pd = find_base(b.row_base, b.count, grow);
        if (pd != stats_pd) {
            // Counts are kept per work-group and written once per problem it worked on.
            if (tid == 0 && stats_pd >= 0) flush_stats<L>(b.probs[stats_pd], s_tests, s_removed);
            stats_pd = pd;
        }
        const Prob &P = b.probs[pd];
        const int64_t n = P.n, W = P.W;
        const int row = (int)(grow - b.row_base[pd]);
        const T *C = static_cast<const T *>(P.C);
        unsigned long long *adj_row = P.adj + (int64_t)row * W;
        if (grow != staged) {
            d = P.deg[row];
            const bool nb_lds = d <= kDcap;
            const bool blk_lds = nb_lds && (long long)d * d <= blk_cap;
            if (nb_lds)
                for (int p = tid; p < d; p += kLevelThreads) {
                    const int k = P.nbr[(int64_t)row * n + p];
                    lds_nb[p] = k;
                    lds_ci[p] = C[(int64_t)row * n + k];
                }
            __syncthreads();
            if (blk_lds) {
                // C[N_i, N_i]: each thread issues 8 independent gathers before storing any.
                const int dd = d * d;
                for (int e0 = tid; e0 < dd; e0 += 8 * kLevelThreads) {
                    T v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int e = e0 + u * kLevelThreads;
                        v[u] = (T)0;
                        if (e < dd) {
                            const int p = e / d, q = e - p * d;
                            v[u] = C[(int64_t)lds_nb[p] * n + lds_nb[q]];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int e = e0 + u * kLevelThreads;
                        if (e < dd) lds_blk[e] = v[u];
                    }
                }
            }
            if (tid == 0) s_mode = (nb_lds ? 1 : 0) | (blk_lds ? 2 : 0) | (W <= kWcap ? 4 : 0);
            staged = grow;
        }
        // Live bits of row i, refreshed at every item (other rows remove edges meanwhile).
        if (W <= kWcap)
            for (int w = tid; w < W; w += kLevelThreads) lds_live[w] = live_word(adj_row + w);
        __syncthreads();
        const int mode = s_mode;
        const int *nbg = P.nbr + (int64_t)row * n;
        auto NB = [&](int p) -> int { return (mode & 1) ? lds_nb[p] : nbg[p]; };
        auto CI = [&](int p) -> T { return (mode & 1) ? lds_ci[p] : C[(int64_t)row * n + nbg[p]]; };
        auto CS = [&](int p, int q) -> T {
            if (p == q) return (T)1;
            return (mode & 2) ? lds_blk[p * d + q] : C[(int64_t)NB(p) * n + NB(q)];
        };
        auto LIVE = [&](int j) -> bool {
            const unsigned long long wv = (mode & 4) ? lds_live[j >> 6] : live_word(adj_row + (j >> 6));
            return (wv >> (j & 63)) & 1ull;
        };
        const double tau = P.tau[L];
        const float tl = P.t[L], band = P.band[L];

        const unsigned long long nS = binom(d, L);
        const long long r0 = s_r0;
        const long long r1 = (long long)nS < r0 + R ? (long long)nS : r0 + R;
        const long long nr = r1 - r0;
        int split, qn, slice;
        long long my_t, my_end;
        if (nr >= kLevelThreads) {
            split = 1;
            slice = 0;
            qn = (int)((nr + kLevelThreads - 1) / kLevelThreads);
            my_t = r0 + (long long)tid * qn;
            my_end = my_t + qn < r1 ? my_t + qn : r1;
        } else {
            // Fewer sets than threads: several threads share one S and split its j loop.
            split = 1;
            while (split * 2 * nr <= kLevelThreads) split *= 2;
            slice = tid % split;
            qn = 1;
            my_t = r0 + tid / split;
            my_end = my_t < r1 ? my_t + 1 : my_t;
        }
        const int psteps = (d + split - 1) / split;
        int since_refresh = 0;

        int P_[L];
#pragma unroll
        for (int c = 0; c < L; ++c) P_[c] = 0;
        for (int step = 0; step < qn; ++step) {
            const long long t = my_t + step;
            if (t >= my_end) break;
            if (step == 0) comb_unrank<L>(d, (unsigned long long)t, P_, binom);
            else comb_next<L>(d, P_);

            // Shared per-S work: Cholesky of M2 = C[S,S], y = L^-1 C[S,i]^T, H11 = 1 - y.y.
            SetFactor<T, L> f;
            f.build(P_, CS, CI);
            int sid[L];
#pragma unroll
            for (int c = 0; c < L; ++c) sid[c] = NB(P_[c]);

            for (int pp = 0; pp < psteps; ++pp) {
                const int p = pp * split + slice;
                if (p >= d) break;
                bool inS = false;
#pragma unroll
                for (int c = 0; c < L; ++c) inS |= P_[c] == p;
                if (inS) continue;
                const int j = NB(p);
                if ((mode & 4) && ++since_refresh >= 16) {
                    // Fold in removals made by other work-groups since the row was staged.
                    since_refresh = 0;
                    atomicAnd(&lds_live[j >> 6], live_word(adj_row + (j >> 6)));
                }
                if (!LIVE(j)) continue;
                ++my_tests;
                const int dec = f.test(P_, p, CS, CI, tau, tl, band);
                if (sizeof(T) == 4 && b.force_recheck) {
                    push_recheck<L>(b, pd, row, j, sid, dec);
                    continue;
                }
                if (dec == 2) {
                    push_recheck<L>(b, pd, row, j, sid, 2);
                } else if (dec == 1) {
                    const int slot = atomicAdd(&s_nstage, 1);
                    if (slot < kStageCap) {
                        s_stage_j[slot] = j;
                        s_stage_t[slot] = (unsigned long long)t;
                    } else {
                        const int lo = row < j ? row : j, hi = row < j ? j : row;
                        if (take_edge(P.adj, W, lo, hi)) {
                            ++my_removed;
                            write_record(P, lo, hi, L, sid);
                        }
                    }
                    if (mode & 4) atomicAnd(&lds_live[j >> 6], ~(1ull << (j & 63)));
                }
            }
        }
        // Settle the staged removals: every ticket is taken at once (one thread each), the
        // winners get consecutive SepSet slots from one atomic add, and re-derive S from its rank.
        __syncthreads();
        const int nst = s_nstage < kStageCap ? s_nstage : kStageCap;
        if (nst > 0) {
            int myslot = -1, sj = 0;
            unsigned long long srank = 0;
            if (tid < nst) {
                sj = s_stage_j[tid];
                srank = s_stage_t[tid];
                const int lo = row < sj ? row : sj, hi = row < sj ? sj : row;
                if (take_edge(P.adj, W, lo, hi)) {
                    ++my_removed;
                    myslot = atomicAdd(&s_nwin, 1);
                }
            }
            __syncthreads();
            if (tid == 0) {
                const int nw = s_nwin;
                s_rec_base = nw ? atomicAdd(reinterpret_cast<unsigned long long *>(P.rec_count),
                                            (unsigned long long)nw)
                                : 0ull;
            }
            __syncthreads();
            if (tid == 0) {
                s_nstage = 0;
                s_nwin = 0;
            }
            if (myslot >= 0) {
                const long long k = (long long)(s_rec_base + (unsigned long long)myslot);
                if (k < P.rec_cap) {
                    int Q[L];
                    comb_unrank<L>(d, srank, Q, binom);
                    int qs[L];
#pragma unroll
                    for (int c = 0; c < L; ++c) qs[c] = NB(Q[c]);
                    store_record(P.recs + k, row < sj ? row : sj, row < sj ? sj : row, L, qs);
                }
            }
        }
        // Per-wavefront sums into the work-group counters of this problem.
        const long long wt = wave_sum_ll(my_tests), wr = wave_sum_ll(my_removed);
        if ((tid & 63) == 0) {
            if (wt) add_ll(&s_tests, wt);
            if (wr) add_ll(&s_removed, wr);
        }
        my_tests = 0;
        my_removed = 0;
    }
    if (tid == 0 && stats_pd >= 0) flush_stats<L>(b.probs[stats_pd], s_tests, s_removed);
}

// ---------------------------------------------------------------------------------------------
// Deep levels (l > kFastLevels): one conditioning set per wavefront
// ---------------------------------------------------------------------------------------------
constexpr int kDeepWaves = kLevelThreads / 64;

// Orders the LDS accesses of the lanes of one wavefront around a cooperative step.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Same work items as k_level (rows and ranges of conditioning-set ranks), but a register-resident
// factor per thread does not fit beyond kFastLevels, so each wavefront takes one set S at a time:
// M2 = C[S,S] is staged in LDS and factored (FP64 Cholesky, lanes splitting each column and the
// trailing update), y = L^-1 C[S,i] and H11 follow, and the lanes then test the candidates j of
// the row against that factor (Eq. 3-6). Tests whose decision the FP32 C leaves open, or whose M2
// has a pivot below the tolerance, go to the FP64 re-check queue.
template <typename T, int L>
__global__ __launch_bounds__(kLevelThreads) void k_level_deep(Batch b, int R) {
    __shared__ long long s_grow, s_r0;
    __shared__ long long s_tests, s_removed;
    __shared__ int s_mode;
    __shared__ int s_nb[kDcap];
    __shared__ T s_ci[kDcap];
    __shared__ unsigned long long s_live[kWcap];
    __shared__ int s_P[kDeepWaves][L];
    __shared__ double s_y[kDeepWaves][L];
    __shared__ double s_M[kDeepWaves][L][L + 1];

    DevState *st = b.st;
    if (st->done) return;
    const unsigned long long total = st->total_items;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const TableBinom binom{b.binom};
    if (tid == 0) { s_tests = 0; s_removed = 0; }
    long long staged = -1, last_row = 0;
    int d = 0, stats_pd = -1;
    long long my_tests = 0, my_removed = 0;
    bool first = true;
    double (*M)[L + 1] = s_M[wave];
    int *PS = s_P[wave];
    double *yv = s_y[wave];

    for (;;) {
        __syncthreads();
        if (tid < 64) {
            unsigned long long g = blockIdx.x;
            if (!first && tid == 0) g = gridDim.x + atomicAdd(&st->next_item, 1ull);
            g = __shfl(g, 0, 64);
            if (g >= total) {
                if (tid == 0) s_grow = -1;
            } else {
                long long lo = last_row, hi = b.total_rows;
                while (hi - lo > 1) {
                    const long long step = (hi - lo + 63) / 64;
                    const long long idx = lo + (long long)tid * step;
                    const bool okb = idx < hi && (unsigned long long)b.item_off[idx] <= g;
                    const unsigned long long mask = __ballot(okb);
                    const int top = 63 - __clzll((long long)mask);
                    lo = lo + (long long)top * step;
                    hi = lo + step < hi ? lo + step : hi;
                }
                if (tid == 0) {
                    s_grow = lo;
                    s_r0 = (long long)(g - (unsigned long long)b.item_off[lo]) * R;
                }
            }
        }
        __syncthreads();
        first = false;
        const long long grow = s_grow;
        if (grow < 0) break;
        last_row = grow;
        const int pd = find_base(b.row_base, b.count, grow);
        if (pd != stats_pd) {
            if (tid == 0 && stats_pd >= 0) flush_stats<L>(b.probs[stats_pd], s_tests, s_removed);
            stats_pd = pd;
        }
        const Prob &P = b.probs[pd];
        const int64_t n = P.n, W = P.W;
        const int row = (int)(grow - b.row_base[pd]);
        const T *C = static_cast<const T *>(P.C);
        unsigned long long *adj_row = P.adj + (int64_t)row * W;
        if (grow != staged) {
            d = P.deg[row];
            const bool nb_lds = d <= kDcap;
            if (nb_lds)
                for (int p = tid; p < d; p += kLevelThreads) {
                    const int k = P.nbr[(int64_t)row * n + p];
                    s_nb[p] = k;
                    s_ci[p] = C[(int64_t)row * n + k];
                }
            if (tid == 0) s_mode = (nb_lds ? 1 : 0) | (W <= kWcap ? 4 : 0);
            staged = grow;
        }
        if (W <= kWcap)
            for (int w = tid; w < W; w += kLevelThreads) s_live[w] = live_word(adj_row + w);
        __syncthreads();
        const int mode = s_mode;
        const int *nbg = P.nbr + (int64_t)row * n;
        auto NB = [&](int p) -> int { return (mode & 1) ? s_nb[p] : nbg[p]; };
        auto CI = [&](int p) -> double { return (double)((mode & 1) ? s_ci[p] : C[(int64_t)row * n + nbg[p]]); };
        auto CS = [&](int p, int q) -> double { return p == q ? 1.0 : (double)C[(int64_t)NB(p) * n + NB(q)]; };
        auto LIVE = [&](int j) -> bool {
            const unsigned long long wv = (mode & 4) ? s_live[j >> 6] : live_word(adj_row + (j >> 6));
            return (wv >> (j & 63)) & 1ull;
        };
        const double tau = P.tau[L];
        const double tl = tanh(tau);
        const double band = (double)P.band[L];
        const double tol = sizeof(T) == 8 ? 1e-12 : 1e-4;

        const unsigned long long nS = binom(d, L);
        const long long r0 = s_r0;
        const long long r1 = (long long)nS < r0 + R ? (long long)nS : r0 + R;
        for (long long t = r0 + wave; t < r1; t += kDeepWaves) {
            int Q[L];
            comb_unrank<L>(d, (unsigned long long)t, Q, binom);
            if (lane == 0) {
#pragma unroll
                for (int c = 0; c < L; ++c) PS[c] = Q[c];
            }
            wave_sync();
            for (int e = lane; e < L * L; e += 64) {
                const int r = e / L, c = e - r * L;
                if (c <= r) M[r][c] = CS(PS[r], PS[c]);
            }
            wave_sync();
            // Right-looking Cholesky in place (lower triangle).
            bool ok = true;
            for (int c = 0; c < L; ++c) {
                const double piv = M[c][c];
                ok = ok && piv > tol;
                const double pv = piv > tol ? piv : 1.0;
                const double rd = 1.0 / sqrt(pv);
                wave_sync();
                if (lane == 0) M[c][c] = sqrt(pv);
                for (int r = c + 1 + lane; r < L; r += 64) M[r][c] *= rd;
                wave_sync();
                const int q = L - c - 1;
                for (int e = lane; e < q * q; e += 64) {
                    const int r = c + 1 + e / q, k = c + 1 + e % q;
                    if (k <= r) M[r][k] -= M[r][c] * M[k][c];
                }
                wave_sync();
            }
            // X = L^-1 by columns (lane k solves L x = e_k), written over the factor; its squared
            // Frobenius norm is tr(M2^-1) for the FP32 error factor g = 1 + sqrt(l tr(M2^-1)).
            double tr = 0.0;
            {
                double x[L];
#pragma unroll
                for (int r = 0; r < L; ++r) {
                    double a = r == lane ? 1.0 : 0.0;
#pragma unroll
                    for (int e = 0; e < r; ++e) a -= M[r][e] * x[e];
                    x[r] = lane < L ? a / M[r][r] : 0.0;
                    tr += x[r] * x[r];
                }
                wave_sync();
                if (lane < L) {
#pragma unroll
                    for (int r = 0; r < L; ++r)
                        if (r >= lane) M[r][lane] = x[r];
                }
                wave_sync();
            }
            tr = wave_sum64(tr);
            const double gf = 1.0 + sqrt((double)L * tr);
            const double g2 = sizeof(T) == 4 ? gf * gf : 4.0;
            // y = X C[S,i] (lane r takes row r), H11 = 1 - |y|^2.
            if (lane < L) {
                double a = 0.0;
                for (int e = 0; e <= lane; ++e) a += M[lane][e] * CI(PS[e]);
                yv[lane] = a;
            }
            wave_sync();
            double yy = 0.0;
            for (int r = 0; r < L; ++r) yy += yv[r] * yv[r];
            const double h11 = 1.0 - yy;
            for (int p = lane; p < d; p += 64) {
                bool inS = false;
#pragma unroll
                for (int c = 0; c < L; ++c) inS |= Q[c] == p;
                if (inS) continue;
                const int j = NB(p);
                if (!LIVE(j)) continue;
                ++my_tests;
                // w = X C[S,j] row by row: H22 = 1 - |w|^2, H12 = C_ij - y.w.
                T cj[L];
#pragma unroll
                for (int e = 0; e < L; ++e) cj[e] = (T)CS(p, Q[e]);
                double ww = 0.0, yw = 0.0;
#pragma unroll
                for (int r = 0; r < L; ++r) {
                    double a = 0.0;
#pragma unroll
                    for (int e = 0; e <= r; ++e) a += M[r][e] * (double)cj[e];
                    ww += a * a;
                    yw += yv[r] * a;
                }
                const double h22 = 1.0 - ww, h12 = CI(p) - yw;
                int dec;
                if (!ok) {
                    dec = 2;
                } else if (sizeof(T) == 8) {
                    const double rho = (h11 > 0.0 && h22 > 0.0) ? h12 / sqrt(h11 * h22) : 0.0;
                    dec = fisher_z64(rho) <= tau ? 1 : 0;
                } else {
                    // FP64 arithmetic on FP32 entries of C: the band only covers C's own error.
                    const double fl = 2.0 * band * g2;
                    if (h11 <= fl || h22 <= fl) {
                        dec = 2;
                    } else {
                        const double inv = 1.0 / sqrt(h11 * h22), ar = fabs(h12) * inv;
                        const double err = band * g2 * (inv + 0.5 * ar * (1.0 / h11 + 1.0 / h22));
                        dec = ar <= tl - err ? 1 : (ar > tl + err ? 0 : 2);
                    }
                }
                if (dec == 1 && !(sizeof(T) == 4 && b.force_recheck)) {
                    const int lo = row < j ? row : j, hi = row < j ? j : row;
                    if (take_edge(P.adj, W, lo, hi)) {
                        int sid[L];
#pragma unroll
                        for (int c = 0; c < L; ++c) sid[c] = NB(Q[c]);
                        ++my_removed;
                        write_record(P, lo, hi, L, sid);
                    }
                    if (mode & 4) atomicAnd(&s_live[j >> 6], ~(1ull << (j & 63)));
                } else if (dec == 2 || (sizeof(T) == 4 && b.force_recheck)) {
                    int sid[L];
#pragma unroll
                    for (int c = 0; c < L; ++c) sid[c] = NB(Q[c]);
                    push_recheck<L>(b, pd, row, j, sid, dec);
                }
            }
            wave_sync();
        }
        const long long wt = wave_sum_ll(my_tests), wr = wave_sum_ll(my_removed);
        if (lane == 0) {
            if (wt) add_ll(&s_tests, wt);
            if (wr) add_ll(&s_removed, wr);
        }
        my_tests = 0;
        my_removed = 0;
    }
    if (tid == 0 && stats_pd >= 0) flush_stats<L>(b.probs[stats_pd], s_tests, s_removed);
}

template <typename T, int L>
static hipError_t launch_level_t(hipStream_t s, const Batch &b, int R, int lds_bytes, int grid) {
    if constexpr (L <= kFastLevels)
        hipLaunchKernelGGL((k_level<T, L>), dim3(grid), dim3(kLevelThreads), lds_bytes, s, b, R, lds_bytes);
    else
        hipLaunchKernelGGL((k_level_deep<T, L>), dim3(grid), dim3(kLevelThreads), 0, s, b, R);
    return hipGetLastError();
}

template <typename T, int L>
struct LevelDispatch {
    static hipError_t run(hipStream_t s, const Batch &b, int level, int R, int lds, int grid) {
        if (level == L) return launch_level_t<T, L>(s, b, R, lds, grid);
        return LevelDispatch<T, L + 1>::run(s, b, level, R, lds, grid);
    }
};
template <typename T>
struct LevelDispatch<T, PC_MAX_LEVEL + 1> {
    static hipError_t run(hipStream_t, const Batch &, int, int, int, int) { return hipErrorInvalidValue; }
};

size_t level_lds_fixed(int prec) {
    return prec == PC_PREC_FP64 ? lds_fixed_bytes<double>() : lds_fixed_bytes<float>();
}

hipError_t launch_level(hipStream_t s, const Batch &b, int level, int R, int lds_bytes, int grid) {
    if (level < 1 || level > PC_MAX_LEVEL) return hipErrorInvalidValue;
    if (b.prec == PC_PREC_FP64) return LevelDispatch<double, 1>::run(s, b, level, R, lds_bytes, grid);
    return LevelDispatch<float, 1>::run(s, b, level, R, lds_bytes, grid);
}

// ---------------------------------------------------------------------------------------------
// FP64 re-check
// ---------------------------------------------------------------------------------------------
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kRcThreads = 256;            // re-check work-group: 4 wavefronts per queued test
constexpr int kRcChunk = 16;               // consecutive samples per lane per round
constexpr int kRcRound = kRcThreads / 16 * kRcChunk;   // samples per round of a work-group (256)

// Statistics of the re-checks a worker settled, written once per problem.
struct RcStats {
    int cur = -1;
    long long rc = 0, rm = 0, viol = 0;
    __device__ void flush(const Batch &b, int l) {
        if (cur < 0) return;
        Prob &Pc = b.probs[cur];
        add_ll(&Pc.rechecks[l], rc);
        if (rm) add_ll(&Pc.removed[l], rm);
        if (viol) add_ll(&Pc.audit_viol[l], viol);
        rc = rm = viol = 0;
    }
    __device__ void at(const Batch &b, int l, int prob) {
        if (prob != cur) {
            flush(b, l);
            cur = prob;
        }
    }
};

// Decision and removal of one re-checked test from its FP64 Gram block G (row stride ld).
__device__ inline void settle_recheck(const Batch &b, Prob &P, int l, const double *G, int ld, double *work,
                                      int mm, int i, int j, int cls, const int *S, RcStats &rs) {
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    const int res = decide_gram64(G, ld, l, P.tau[l], work, mm);
    ++rs.rc;
    if (b.force_recheck && cls != 2 && cls != res) ++rs.viol;
    // The atomic on the canonical bit decides: an edge another test already removed stays
    // removed and keeps that test's SepSet.
    if (res && take_edge(P.adj, P.W, lo, hi)) {
        ++rs.rm;
        write_record(P, lo, hi, l, S);
    }
}

// Queued tests of levels up to 14 (at most 16 variables): one wavefront per test, grid-stride.
// The FP64 Gram block of the standardized rows (i, j, S) is one 16 x 16 tile Z Z^T accumulated
// on v_mfma_f64_16x16x4f64 over all samples: lane l carries row l % 16 (so the same register is
// both the A operand, Z, and the B operand, Z^T) and 16 consecutive samples per round; each k-step
// sums four samples. Rows past l + 2 stay zero. On the FP64 path the block is read from C.
__global__ __launch_bounds__(kRcThreads) void k_recheck(Batch b, int level) {
    constexpr int kW = kRcThreads / 64;
    __shared__ double G[kW][16 * 16];
    __shared__ double work[kW][kWorks];
    __shared__ int s_v[kW][16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned long long pushed = b.st->rq_count;
    const long long count = pushed < (unsigned long long)b.rq_cap ? (long long)pushed : b.rq_cap;
    const int l = level, k = l + 2;
    double *Gw = G[wave];
    int *vw = s_v[wave];
    RcStats rs;
    for (long long e = (long long)blockIdx.x * kW + wave; e < count; e += (long long)gridDim.x * kW) {
        const RqEntry *qe = b.rq + e;
        if (lane < 16) vw[lane] = lane == 0 ? qe->i : (lane == 1 ? qe->j : (lane < k ? (int)qe->S[lane - 2] : -1));
        const int prob = qe->prob, cls = qe->cls;
        wave_sync();
        Prob &P = b.probs[prob];
        if (b.prec != PC_PREC_FP64) {
            const int64_t mp = P.mp;
            const int vr = vw[lane & 15];
            const double *z = P.zt64 + (int64_t)(vr < 0 ? 0 : vr) * mp;
            const int64_t off = (int64_t)(lane >> 4) * kRcChunk;
            doublex4 acc = {0.0, 0.0, 0.0, 0.0};
            // Four rounds of 64 samples per step, all loads issued before their products. mp is
            // a multiple of 64, so a lane's chunk of 16 is either wholly inside or outside.
            for (int64_t x0 = 0; x0 < mp; x0 += 4 * 64) {
                double v[4][kRcChunk];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t x = x0 + 64 * q + off;
                    if (vr >= 0 && x < mp) {
                        const double2 *src = reinterpret_cast<const double2 *>(z + x);
#pragma unroll
                        for (int u = 0; u < kRcChunk / 2; ++u) {
                            const double2 t = src[u];
                            v[q][2 * u] = t.x;
                            v[q][2 * u + 1] = t.y;
                        }
                    } else {
#pragma unroll
                        for (int u = 0; u < kRcChunk; ++u) v[q][u] = 0.0;
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int u = 0; u < kRcChunk; ++u)
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(v[q][u], v[q][u], acc, 0, 0, 0);
            }
            // D layout of the FP64 16x16x4 product: lane l holds rows l / 16 + 4 t, column l % 16.
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
        if (lane == 0) {
            rs.at(b, l, prob);
            settle_recheck(b, P, l, Gw, 16, work[wave], kMMs, vw[0], vw[1], cls, vw + 2, rs);
        }
        wave_sync();
    }
    if (lane == 0) rs.flush(b, l);
}

// Queued tests of deeper levels (17 to 32 variables): one work-group per test. The Gram block
// spans 2 x 2 tiles of 16 x 16; wavefront w accumulates tile (w / 2, w % 2) over all samples.
__global__ __launch_bounds__(kRcThreads) void k_recheck_deep(Batch b, int level) {
    __shared__ double part[kRcThreads / 64][16 * 16];
    __shared__ double G[kGramLd * kGramLd];
    __shared__ double work[kWork];
    __shared__ int s_v[32];        // variables of the tile rows: i, j, S..., then -1
    __shared__ int s_prob, s_cls;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned long long pushed = b.st->rq_count;
    const long long count = pushed < (unsigned long long)b.rq_cap ? (long long)pushed : b.rq_cap;
    const int l = level, k = l + 2;
    RcStats rs;
    for (long long e = blockIdx.x; e < count; e += gridDim.x) {
        const RqEntry *qe = b.rq + e;
        if (tid < 32) s_v[tid] = tid == 0 ? qe->i : (tid == 1 ? qe->j : (tid < k ? (int)qe->S[tid - 2] : -1));
        if (tid == 0) {
            s_prob = qe->prob;
            s_cls = qe->cls;
        }
        __syncthreads();
        const int prob = s_prob;
        Prob &P = b.probs[prob];
        if (b.prec != PC_PREC_FP64) {
            const int64_t mp = P.mp;
            const int ra = s_v[16 * (wave >> 1) + (lane & 15)], rb = s_v[16 * (wave & 1) + (lane & 15)];
            const double *za = P.zt64 + (int64_t)(ra < 0 ? 0 : ra) * mp;
            const double *zb = P.zt64 + (int64_t)(rb < 0 ? 0 : rb) * mp;
            const int64_t off = (int64_t)(lane >> 4) * kRcChunk;
            doublex4 acc = {0.0, 0.0, 0.0, 0.0};
            for (int64_t x0 = 0; x0 < mp; x0 += 4 * kRcChunk) {
                const int64_t x = x0 + off;
                double va[kRcChunk], vb[kRcChunk];
#pragma unroll
                for (int u = 0; u < kRcChunk; ++u) {
                    va[u] = ra >= 0 && x < mp ? za[x + u] : 0.0;
                    vb[u] = rb >= 0 && x < mp ? zb[x + u] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < kRcChunk; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va[u], vb[u], acc, 0, 0, 0);
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) part[wave][((lane >> 4) + 4 * t) * 16 + (lane & 15)] = acc[t];
            __syncthreads();
            for (int q = tid; q < 4 * 256; q += kRcThreads) {
                const int w = q >> 8, rr = 16 * (w >> 1) + ((q & 255) >> 4), cc = 16 * (w & 1) + (q & 15);
                if (rr < k && cc < k) G[rr * kGramLd + cc] = rr == cc ? 1.0 : part[w][q & 255];
            }
        } else {
            for (int q = tid; q < k * k; q += kRcThreads) {
                const int rr = q / k, cc = q % k;
                G[rr * kGramLd + cc] = rr == cc ? 1.0 : static_cast<const double *>(P.C)[(int64_t)s_v[rr] * P.n + s_v[cc]];
            }
        }
        __syncthreads();
        if (tid == 0) {
            rs.at(b, l, prob);
            settle_recheck(b, P, l, G, kGramLd, work, kMM, s_v[0], s_v[1], s_cls, s_v + 2, rs);
        }
        __syncthreads();
    }
    if (tid == 0) rs.flush(b, l);
}

hipError_t launch_recheck(hipStream_t s, const Batch &b, int level, int grid) {
    if (level + 2 <= 16)
        hipLaunchKernelGGL(k_recheck, dim3(grid), dim3(kRcThreads), 0, s, b, level);
    else
        hipLaunchKernelGGL(k_recheck_deep, dim3(grid), dim3(kRcThreads), 0, s, b, level);
    return hipGetLastError();
}

}  // namespace pcg
