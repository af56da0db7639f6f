// Levels l >= 1 of PC-stable (Algorithm 1, Sec. 2.4) on gfx950.
//
// k_compact: the snapshot G' := G as compacted neighbour lists (the A'_G of Sec. 3.3 / Fig. 2):
//   one wavefront per row turns the row's bit words into ascending neighbour ids with popcount and
//   a wave prefix sum, then the last work-group to finish scans the per-row work counts into the
//   work plan of the level. A level with no row of degree >= l + 1 sets the device stop flag: that
//   is the max-degree test of Algorithm 2 kept on the device.
//
// k_level<T, L>: the CI tests of level L. A work item is a row i with a range of ranks of its
//   l-subsets S of adj(i, G') (the set-sharing view of cuPC-S, Sec. 3.4): for each S the
//   Cholesky factor of M2 = C[S,S] (Eq. 3) is formed once and serves every j in adj(i,G') \ S, so
//   the per-j work is one triangular solve. The row's neighbour list, C[i, N_i] and (for l >= 2)
//   the block C[N_i, N_i] are staged in LDS once per item. Items come from a device-side queue
//   that a fixed grid of work-groups drains (persistent kernel), absorbing the very uneven
//   per-row subset counts C(d_i, l).
//   Every test first checks that edge (i,j) is still in G (early termination, Sec. 4.1). The first
//   independent test clears the edge with an atomic AND on the bit (min, max); only the thread
//   whose AND cleared it writes the SepSet record, so each removed edge has exactly one record.
//   FP32 tests whose |rho| lies within an error band of tanh(tau_l) (and FP64 tests whose M2 is
//   rank deficient) go to a re-check queue.
//
// k_recheck: one wavefront per queued test re-evaluates it in FP64 (the block of C recomputed as
//   dot products of the FP64 standardized columns, or read from the FP64 C), with a
//   pseudo-inverse when M2 is rank deficient, and removes the edge if that decides independence.
#include "pc_comb.h"
#include "pc_dev.h"

namespace pcg {

__device__ inline double wave_sum64(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline double fisher_z64(double r) {
    if (!(fabs(r) < 1.0)) return INFINITY;
    return fabs(0.5 * log((1.0 + r) / (1.0 - r)));
}

__device__ inline unsigned long long live_word(unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline long long load_ll(const long long *p) {
    return __hip_atomic_load(const_cast<long long *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------------------------
// Compaction and planning
// ---------------------------------------------------------------------------------------------
constexpr unsigned long long kMaxSetsPerRow = 1ull << 40;

__global__ __launch_bounds__(256) void k_compact(const unsigned long long *__restrict__ adj,
                                                 int64_t n, int64_t W, int level, int R,
                                                 int *__restrict__ nbr, int *__restrict__ deg,
                                                 long long *nitems, long long *item_off,
                                                 const unsigned long long *__restrict__ binom,
                                                 DevState *st) {
    __shared__ int is_last;
    __shared__ long long part[256];
    if (st->done) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t i = (int64_t)blockIdx.x * 4 + wave;
    if (i < n) {
        const unsigned long long *row = adj + i * W;
        int *out = nbr + i * n;
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
                int t = __shfl_up(incl, o, 64);
                if (lane >= o) incl += t;
            }
            const int tot = __shfl(incl, 63, 64);
            int pos = count + incl - pc;
            while (word) {
                const int b = __ffsll((long long)word) - 1;
                out[pos++] = (int)(w * 64 + b);
                word &= word - 1;
            }
            count += tot;
        }
        if (lane == 0) {
            deg[i] = count;
            atomicMax(&st->deg_work, count);
            long long items = 0;
            if (count >= level + 1) {
                const unsigned long long nS = binom[(int64_t)count * kBinomCols + level];
                if (nS > kMaxSetsPerRow) {
                    atomicOr(&st->overflow, 1);
                } else {
                    items = (long long)((nS + (unsigned long long)R - 1) / (unsigned long long)R);
                }
            }
            nitems[i] = items;
        }
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) is_last = atomicAdd(&st->blocks_done, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    const int64_t chunk = (n + 255) / 256;
    const int64_t lo = tid * chunk, hi = lo + chunk < n ? lo + chunk : n;
    long long s = 0;
    for (int64_t k = lo; k < hi; ++k) s += load_ll(nitems + k);
    part[tid] = s;
    __syncthreads();
    if (tid == 0) {
        long long run = 0;
        for (int k = 0; k < 256; ++k) {
            long long v = part[k];
            part[k] = run;
            run += v;
        }
        item_off[n] = run;
        const int md = __hip_atomic_load(&st->deg_work, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        st->max_deg = md;
        st->maxdeg[level] = md;
        st->total_items = (unsigned long long)run;
        st->items[level] = run;
        st->next_item = 0ull;
        st->rq_count = 0ull;
        st->deg_work = 0;
        st->blocks_done = 0u;
        if (run == 0) st->done = 1;
    }
    __syncthreads();
    long long run = part[tid];
    for (int64_t k = lo; k < hi; ++k) {
        item_off[k] = run;
        run += load_ll(nitems + k);
    }
}

hipError_t launch_compact(hipStream_t s, const unsigned long long *adj, int64_t n, int64_t W,
                          int level, int ranks_per_item, int *nbr, int *deg, long long *nitems,
                          long long *item_off, const unsigned long long *binom, DevState *st) {
    dim3 grid((unsigned)((n + 3) / 4));
    hipLaunchKernelGGL(k_compact, grid, dim3(256), 0, s, adj, n, W, level, ranks_per_item, nbr,
                       deg, nitems, item_off, binom, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// FP64 decision from a Gram block (used by the re-check and by rank-deficient FP64 tests)
// ---------------------------------------------------------------------------------------------

// Per-wave FP64 scratch of the re-check path, kept in LDS (runtime-sized small matrices).
constexpr int kMM = PC_MAX_LEVEL * PC_MAX_LEVEL;
constexpr int kWork = 4 * kMM + 2 * PC_MAX_LEVEL;   // Lm, a, v, P, y, w

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
// work: kWork doubles of scratch.
__device__ int decide_gram64(const double *G, int ld, int l, double tau, double *work) {
    double h11 = 1.0, h22 = 1.0, h12 = G[1];
    if (l > 0) {
        double *Lm = work, *a = work + kMM, *v = work + 2 * kMM, *P = work + 3 * kMM;
        double *y = work + 4 * kMM, *w = y + PC_MAX_LEVEL;
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

// Clears edge (lo, hi) from G. Returns true for the one caller whose atomic AND on the canonical
// bit (row lo, column hi) found it set: that caller owns the SepSet record.
__device__ inline bool take_edge(unsigned long long *adj, int64_t W, int lo, int hi) {
    const unsigned long long bit = 1ull << (hi & 63);
    const unsigned long long old = atomicAnd(adj + (int64_t)lo * W + (hi >> 6), ~bit);
    if (!(old & bit)) return false;
    atomicAnd(adj + (int64_t)hi * W + (lo >> 6), ~(1ull << (lo & 63)));
    return true;
}

// ---------------------------------------------------------------------------------------------
// Level kernel
// ---------------------------------------------------------------------------------------------
constexpr int kDcap = 1024;  // neighbour lists up to this degree are staged in LDS

struct TableBinom {
    const unsigned long long *t;
    __device__ unsigned long long operator()(int a, int b) const {
        if (b < 0 || a < b) return 0ull;
        return t[(int64_t)a * kBinomCols + b];
    }
};

template <typename T>
__host__ __device__ constexpr size_t lds_fixed_bytes() {
    return (sizeof(int) * kDcap + 15) / 16 * 16 + (sizeof(T) * kDcap + 15) / 16 * 16;
}

// Pushes a test to the re-check queue; cls is the FP32 classification (0 dependent, 1 independent,
// 2 inside the band).
template <int L>
__device__ inline void push_recheck(const LevelArgs &a, int row, int j, const int (&sid)[L], int cls) {
    const unsigned long long k = atomicAdd(&a.st->rq_count, 1ull);
    if (k >= (unsigned long long)a.rq_cap) {
        atomicOr(&a.st->rq_overflow, 1);
        return;
    }
    pc_sep_rec *e = a.rq + k;
    e->i = row;
    e->j = j;
    e->level = cls;
#pragma unroll
    for (int c = 0; c < PC_MAX_LEVEL; ++c) e->S[c] = c < L ? sid[c] : -1;
}

template <typename T, int L>
__global__ __launch_bounds__(kLevelThreads) void k_level(LevelArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_row;
    __shared__ long long s_r0;
    __shared__ int s_mode;  // bit 0: nb/ci in LDS, bit 1: C[N_i,N_i] in LDS
    __shared__ long long s_tests, s_removed;

    DevState *st = a.st;
    if (st->done) return;
    const unsigned long long total = st->total_items;
    const int tid = threadIdx.x;
    int *lds_nb = reinterpret_cast<int *>(smem);
    T *lds_ci = reinterpret_cast<T *>(smem + (sizeof(int) * kDcap + 15) / 16 * 16);
    T *lds_blk = reinterpret_cast<T *>(smem + lds_fixed_bytes<T>());
    const long long blk_cap = ((long long)a.lds_bytes - (long long)lds_fixed_bytes<T>()) / (long long)sizeof(T);
    const T *C = static_cast<const T *>(a.C);
    const TableBinom binom{a.binom};
    const int64_t n = a.n, W = a.W;

    if (tid == 0) { s_tests = 0; s_removed = 0; }
    int staged = -1, last_row = 0, d = 0;
    long long my_tests = 0, my_removed = 0;

    for (;;) {
        __syncthreads();
        if (tid == 0) {
            const unsigned long long g = atomicAdd(&st->next_item, 1ull);
            if (g >= total) {
                s_row = -1;
            } else {
                int lo = last_row, hi = (int)n;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if ((unsigned long long)a.item_off[mid] <= g) lo = mid; else hi = mid;
                }
                s_row = lo;
                s_r0 = (long long)(g - (unsigned long long)a.item_off[lo]) * a.ranks_per_item;
            }
        }
        __syncthreads();
        const int row = s_row;
        if (row < 0) break;
        last_row = row;
        if (row != staged) {
            d = a.deg[row];
            const bool nb_lds = d <= kDcap;
            const bool blk_lds = nb_lds && L >= 2 && (long long)d * d <= blk_cap;
            if (nb_lds)
                for (int p = tid; p < d; p += kLevelThreads) {
                    const int k = a.nbr[(int64_t)row * n + p];
                    lds_nb[p] = k;
                    lds_ci[p] = C[(int64_t)row * n + k];
                }
            __syncthreads();
            if (blk_lds)
                for (int e = tid; e < d * d; e += kLevelThreads) {
                    const int p = e / d, q = e - p * d;
                    lds_blk[e] = C[(int64_t)lds_nb[p] * n + lds_nb[q]];
                }
            if (tid == 0) s_mode = (nb_lds ? 1 : 0) | (blk_lds ? 2 : 0);
            staged = row;
            __syncthreads();
        }
        const int mode = s_mode;
        const int *nbg = a.nbr + (int64_t)row * n;
        auto NB = [&](int p) -> int { return (mode & 1) ? lds_nb[p] : nbg[p]; };
        auto CI = [&](int p) -> T { return (mode & 1) ? lds_ci[p] : C[(int64_t)row * n + nbg[p]]; };
        auto CS = [&](int p, int q) -> T {
            if (p == q) return (T)1;
            return (mode & 2) ? lds_blk[p * d + q] : C[(int64_t)NB(p) * n + NB(q)];
        };

        const unsigned long long nS = binom(d, L);
        const long long r0 = s_r0;
        const long long r1 = (long long)nS < r0 + a.ranks_per_item ? (long long)nS : r0 + a.ranks_per_item;
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

        int P[L];
#pragma unroll
        for (int c = 0; c < L; ++c) P[c] = 0;
        for (int step = 0; step < qn; ++step) {
            const long long t = my_t + step;
            if (t >= my_end) break;
            if (step == 0) comb_unrank<L>(d, (unsigned long long)t, P, binom);
            else comb_next<L>(d, P);

            // Shared per-S work: Cholesky of M2 = C[S,S], y = L^-1 C[S,i]^T, H11 = 1 - y.y.
            T Lm[L * (L + 1) / 2];
            T rd[L];
            T y[L];
            bool ok = true;
#pragma unroll
            for (int r = 0; r < L; ++r) {
#pragma unroll
                for (int c = 0; c <= r; ++c) {
                    T s = CS(P[r], P[c]);
#pragma unroll
                    for (int e = 0; e < c; ++e) s -= Lm[r * (r + 1) / 2 + e] * Lm[c * (c + 1) / 2 + e];
                    if (r == c) {
                        const T tol = sizeof(T) == 8 ? (T)1e-12 : (T)1e-4;
                        if (!(s > tol)) ok = false;
                        const T piv = s > tol ? s : (T)1;
                        Lm[r * (r + 1) / 2 + r] = sqrt(piv);
                        rd[r] = (T)1 / sqrt(piv);
                    } else {
                        Lm[r * (r + 1) / 2 + c] = s * rd[c];
                    }
                }
            }
            T yy = 0;
#pragma unroll
            for (int r = 0; r < L; ++r) {
                T s = CI(P[r]);
#pragma unroll
                for (int e = 0; e < r; ++e) s -= Lm[r * (r + 1) / 2 + e] * y[e];
                y[r] = s * rd[r];
                yy += y[r] * y[r];
            }
            const T h11 = (T)1 - yy;
            float g2 = 4.0f;
            if (sizeof(T) == 4 && L > 1) {
                // g = 1 + sqrt(l tr(M2^-1)) bounds 1 + ||M2^-1 c||_1 for any |c| with
                // c^T M2^-1 c <= 1, where tr(M2^-1) = ||L^-1||_F^2.
                float tr = 0.0f;
#pragma unroll
                for (int k = 0; k < L; ++k) {
                    float x[L];
#pragma unroll
                    for (int r = 0; r < L; ++r) {
                        if (r < k) { x[r] = 0.0f; continue; }
                        float s = r == k ? 1.0f : 0.0f;
#pragma unroll
                        for (int e = 0; e < r; ++e) s -= (float)Lm[r * (r + 1) / 2 + e] * x[e];
                        x[r] = s * (float)rd[r];
                        tr += x[r] * x[r];
                    }
                }
                const float g = 1.0f + sqrtf((float)L * tr);
                g2 = g * g;
            }
            int sid[L];
#pragma unroll
            for (int c = 0; c < L; ++c) sid[c] = NB(P[c]);

            for (int pp = 0; pp < psteps; ++pp) {
                const int p = pp * split + slice;
                if (p >= d) break;
                bool inS = false;
#pragma unroll
                for (int c = 0; c < L; ++c) inS |= P[c] == p;
                if (inS) continue;
                const int j = NB(p);
                const unsigned long long wv = live_word(a.adj + (int64_t)row * W + (j >> 6));
                if (!((wv >> (j & 63)) & 1ull)) continue;
                ++my_tests;
                T w[L];
                T ww = 0, yw = 0;
#pragma unroll
                for (int r = 0; r < L; ++r) {
                    T s = CS(p, P[r]);
#pragma unroll
                    for (int e = 0; e < r; ++e) s -= Lm[r * (r + 1) / 2 + e] * w[e];
                    w[r] = s * rd[r];
                    ww += w[r] * w[r];
                    yw += y[r] * w[r];
                }
                const T h22 = (T)1 - ww;
                const T h12 = CI(p) - yw;
                int dec;  // 0 dependent, 1 independent, 2 re-check in FP64
                if (sizeof(T) == 8) {
                    if (ok) {
                        const double rho = (h11 > 0 && h22 > 0) ? (double)h12 / sqrt((double)h11 * (double)h22) : 0.0;
                        dec = fisher_z64(rho) <= a.tau ? 1 : 0;
                    } else {
                        dec = 2;  // rank-deficient M2: pseudo-inverse path of the re-check kernel
                    }
                } else {
                    const float fh11 = (float)h11, fh22 = (float)h22;
                    const float floor_ = 2.0f * a.band * g2;
                    if (!ok || fh11 <= floor_ || fh22 <= floor_) {
                        dec = 2;
                    } else {
                        const float inv = rsqrtf(fh11 * fh22);
                        const float ar = fabsf((float)h12 * inv);
                        const float err = a.band * g2 * (inv + 0.5f * ar * (1.0f / fh11 + 1.0f / fh22));
                        dec = ar <= a.t - err ? 1 : (ar > a.t + err ? 0 : 2);
                    }
                    if (a.force_recheck) {
                        push_recheck<L>(a, row, j, sid, dec);
                        continue;
                    }
                }
                if (dec == 2) {
                    push_recheck<L>(a, row, j, sid, 2);
                } else if (dec == 1) {
                    const int lo = row < j ? row : j, hi = row < j ? j : row;
                    if (take_edge(a.adj, W, lo, hi)) {
                        ++my_removed;
                        const long long k = (long long)atomicAdd((unsigned long long *)a.rec_count, 1ull);
                        if (k < a.rec_cap) {
                            pc_sep_rec *rec = a.recs + k;
                            rec->i = lo;
                            rec->j = hi;
                            rec->level = L;
#pragma unroll
                            for (int c = 0; c < PC_MAX_LEVEL; ++c) rec->S[c] = c < L ? sid[c] : -1;
                        }
                    }
                }
            }
        }
    }
    if (my_tests) add_ll(&s_tests, my_tests);
    if (my_removed) add_ll(&s_removed, my_removed);
    __syncthreads();
    if (tid == 0) {
        if (s_tests) add_ll(&st->tests[L], s_tests);
        if (s_removed) add_ll(&st->removed[L], s_removed);
    }
}

template <typename T, int L>
static hipError_t launch_level_t(hipStream_t s, const LevelArgs &a, int grid) {
    hipLaunchKernelGGL((k_level<T, L>), dim3(grid), dim3(kLevelThreads), a.lds_bytes, s, a);
    return hipGetLastError();
}

template <typename T, int L>
struct LevelDispatch {
    static hipError_t run(hipStream_t s, const LevelArgs &a, int grid) {
        if (a.level == L) return launch_level_t<T, L>(s, a, grid);
        return LevelDispatch<T, L + 1>::run(s, a, grid);
    }
};
template <typename T>
struct LevelDispatch<T, PC_MAX_LEVEL + 1> {
    static hipError_t run(hipStream_t, const LevelArgs &, int) { return hipErrorInvalidValue; }
};

size_t level_lds_fixed(int prec) {
    return prec == PC_PREC_FP64 ? lds_fixed_bytes<double>() : lds_fixed_bytes<float>();
}

hipError_t launch_level(hipStream_t s, const LevelArgs &a, int prec, int grid) {
    if (a.level < 1 || a.level > PC_MAX_LEVEL) return hipErrorInvalidValue;
    if (prec == PC_PREC_FP64) return LevelDispatch<double, 1>::run(s, a, grid);
    return LevelDispatch<float, 1>::run(s, a, grid);
}

// ---------------------------------------------------------------------------------------------
// FP64 re-check
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_recheck(RecheckArgs a) {
    __shared__ double G[4][kGramLd * kGramLd];
    __shared__ double work[4][kWork];
    __shared__ int vl[4][kGramLd];
    __shared__ long long s_rechecks, s_removed, s_viol;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) { s_rechecks = 0; s_removed = 0; s_viol = 0; }
    __syncthreads();
    DevState *st = a.st;
    const unsigned long long pushed = st->rq_count;
    const long long count = pushed < (unsigned long long)a.rq_cap ? (long long)pushed : a.rq_cap;
    const int l = a.level, k = l + 2;
    long long my_rechecks = 0, my_removed = 0, my_viol = 0;
    for (long long e = (long long)blockIdx.x * 4 + wave; e < count; e += (long long)gridDim.x * 4) {
        const pc_sep_rec q = a.rq[e];
        const int i = q.i, j = q.j, cls = q.level;
        const int lo = i < j ? i : j, hi = i < j ? j : i;
        const bool live = (live_word(a.adj + (int64_t)lo * a.W + (hi >> 6)) >> (hi & 63)) & 1ull;
        if (!live && !a.audit) continue;
        if (lane < k) vl[wave][lane] = lane == 0 ? i : (lane == 1 ? j : q.S[lane - 2]);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        double *g = G[wave];
        if (a.zt64) {
            for (int r = 0; r < k; ++r) {
                const double *zr = a.zt64 + (int64_t)vl[wave][r] * a.mp;
                for (int c = r + 1; c < k; ++c) {
                    const double *zc = a.zt64 + (int64_t)vl[wave][c] * a.mp;
                    double s = 0.0;
                    for (int64_t x = lane; x < a.m; x += 64) s += zr[x] * zc[x];
                    s = wave_sum64(s);
                    if (lane == 0) { g[r * kGramLd + c] = s; g[c * kGramLd + r] = s; }
                }
                if (lane == 0) g[r * kGramLd + r] = 1.0;
            }
        } else if (lane == 0) {
            for (int r = 0; r < k; ++r)
                for (int c = 0; c < k; ++c)
                    g[r * kGramLd + c] = r == c ? 1.0 : a.C64[(int64_t)vl[wave][r] * a.n + vl[wave][c]];
        }
        int res = 0;
        if (lane == 0) res = decide_gram64(g, kGramLd, l, a.tau, work[wave]);
        res = __shfl(res, 0, 64);
        if (lane == 0) {
            ++my_rechecks;
            if (a.audit && cls != 2 && cls != res) ++my_viol;
            if (res && live && take_edge(a.adj, a.W, lo, hi)) {
                ++my_removed;
                const long long r = (long long)atomicAdd((unsigned long long *)a.rec_count, 1ull);
                if (r < a.rec_cap) {
                    pc_sep_rec *rec = a.recs + r;
                    rec->i = lo;
                    rec->j = hi;
                    rec->level = l;
                    for (int c = 0; c < PC_MAX_LEVEL; ++c) rec->S[c] = c < l ? q.S[c] : -1;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
    if (lane == 0) {
        if (my_rechecks) add_ll(&s_rechecks, my_rechecks);
        if (my_removed) add_ll(&s_removed, my_removed);
        if (my_viol) add_ll(&s_viol, my_viol);
    }
    __syncthreads();
    if (tid == 0) {
        if (s_rechecks) add_ll(&st->rechecks[l], s_rechecks);
        if (s_removed) add_ll(&st->removed[l], s_removed);
        if (s_viol) add_ll(&st->audit_viol[l], s_viol);
    }
}

hipError_t launch_recheck(hipStream_t s, const RecheckArgs &a, int grid) {
    hipLaunchKernelGGL(k_recheck, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace pcg
