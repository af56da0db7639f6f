// Device code of levels l >= 1 of PC-stable (Algorithm 1, Sec. 2.4) on gfx950, for a batch of problems.
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
// k_recheck: each queued test is re-evaluated in FP64 (the block of C recomputed as dot products
//   of the FP64 standardized columns on FP64 MFMA, or read from the FP64 C) by a wavefront or, when
//   few are queued, a work-group; the S rows are eliminated in registers (a pseudo-inverse when M2
//   is numerically singular), and the edge is removed if that decides independence.
//
// This header holds the kernel templates and their device helpers. The translation units that
// instantiate them are split by type and depth so that the library builds in parallel:
// pc_level_f32.hip and pc_level_f64.hip (k_level, l <= 13), pc_level_deep.hip (k_level_deep),
// pc_recheck.hip (re-check kernels) and pc_level.hip (compaction, planning, dispatch).
#pragma once

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
__device__ inline void flush_stats(const Batch &b, Prob &P, long long &tests, long long &removed) {
    if (tests) add_ll(&P.tests[L], tests);
    if (removed) add_ll(&P.removed[L], removed);
    if (b.probe) {
        if (tests) add_ll(&P.probe_tests[L], tests);
        if (removed) add_ll(&P.probe_removed[L], removed);
    }
    tests = 0;
    removed = 0;
}

// Whether level l runs for problem P (the level cap, Eq. 6 needing m - l - 3 > 0), and was not
// already run by the tail kernel.
__device__ inline bool level_enabled(const Prob &P, int l) {
    return l <= P.max_level && l <= PC_MAX_LEVEL && P.tau[l] == P.tau[l] && l > P.tail_done;
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
__device__ inline void pinv_jacobi(const double *A, int lda, int k, double *a, double *v, double *P) {
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
__device__ inline int decide_gram64(const double *G, int ld, int l, double tau, double *work, int mm) {
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
// FP64 Gram tile of up to 16 standardized variables (re-checks)
// ---------------------------------------------------------------------------------------------
typedef double doublex4 __attribute__((ext_vector_type(4)));
constexpr int kRcChunk = 16;   // consecutive samples per lane per round

// One wavefront's share of the 16 x 16 tile Z Z^T of the FP64 standardized rows vr (lane l
// carries tile row l % 16; vr < 0 gives a zero row), on v_mfma_f64_16x16x4f64: the same register is
// the A operand (Z) and the B operand (Z^T) and each k-step sums four samples. The wavefront takes
// the blocks of 256 samples starting at x_first, x_first + x_step, ...; within a block, lane l
// reads the 16 consecutive samples 64 q + 16 (l / 16) of round q = 0..3, all loads issued before
// the products, and each round feeds its own accumulator so the four product chains overlap.
// Returns the tile in the D layout of the instruction (lane l: rows l / 16 + 4 t, column l % 16).
// R < 4 rounds per block (blocks of 64 R samples) hold fewer samples in registers at once.
template <int R = 4>
__device__ inline doublex4 gram_part(const Prob &P, int vr, int lane, int64_t x_first, int64_t x_step) {
    const int64_t mp = P.mp;
    const double *z = P.zt64 + (int64_t)(vr < 0 ? 0 : vr) * mp;
    const int64_t off = (int64_t)(lane >> 4) * kRcChunk;
    doublex4 acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = doublex4{0.0, 0.0, 0.0, 0.0};
    // mp is a multiple of 64, so a lane's chunk of 16 is either wholly inside or outside.
    for (int64_t x0 = x_first; x0 < mp; x0 += x_step) {
        double v[R][kRcChunk];
#pragma unroll
        for (int q = 0; q < R; ++q) {
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
        for (int u = 0; u < kRcChunk; ++u)
#pragma unroll
            for (int q = 0; q < R; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[q][u], v[q][u], acc[q], 0, 0, 0);
    }
    if constexpr (R == 4) return (acc[0] + acc[1]) + (acc[2] + acc[3]);
    else if constexpr (R == 2) return acc[0] + acc[1];
    else return acc[0];
}

// Broadcast of lane `src`'s double (src uniform) through two scalar reads.
__device__ inline double readlane_f64(double v, int src) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, src);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), src);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// FP64 decision of one test from its Gram block G (rows/columns i, j, S..., K = l + 2 <= KMAX,
// row stride ld, unit diagonal), by a whole wavefront: lane r holds row r in registers and the
// rows of S are eliminated one pivot at a time (symmetric Gaussian elimination, each pivot row
// broadcast from its lane). What is left in rows/columns {i, j} is the Schur complement
// H = M0 - M1 M2^-1 M1^T of Eq. 3, so rho = H12 / sqrt(H11 H22) (Eq. 4). Returns 1 iff
// z(rho) <= tau, 0 if not, and -1 when a pivot is <= 1e-12 (M2 numerically singular: the caller
// takes the pseudo-inverse route). Every lane gets the same result.
template <int KMAX>
__device__ inline int decide_elim(const double *G, int ld, int K, double tau, int lane) {
    double a[KMAX];
#pragma unroll
    for (int c = 0; c < KMAX; ++c) a[c] = (lane < K && c < K) ? G[lane * ld + c] : 0.0;
    bool singular = false;
#pragma unroll
    for (int k = 2; k < KMAX; ++k) {
        if (k < K) {
            const double akk = readlane_f64(a[k], k);
            // The diagonal of M2 is 1, so its Cholesky pivots (these Schur pivots) are compared
            // with 1e-12 times that maximum, as on the pseudo-inverse route.
            singular |= !(akk > 1e-12);
            const double f = a[k] / akk;   // lane r: a_rk / a_kk
#pragma unroll
            for (int c = 0; c < KMAX; ++c)
                if (c < K && (c <= 1 || c > k)) a[c] -= f * readlane_f64(a[c], k);
        }
    }
    if (singular) return -1;
    const double h11 = readlane_f64(a[0], 0), h12 = readlane_f64(a[1], 0), h22 = readlane_f64(a[1], 1);
    const double rho = (h11 > 0.0 && h22 > 0.0) ? h12 / sqrt(h11 * h22) : 0.0;
    return fisher_z64(rho) <= tau ? 1 : 0;
}

// ---------------------------------------------------------------------------------------------
// Re-check helpers (re-check and tail kernels)
// ---------------------------------------------------------------------------------------------
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

// Statistics and removal of one re-checked test with FP64 decision res (one lane).
__device__ inline void settle_recheck(const Batch &b, Prob &P, int l, int res, int i, int j, int cls, const int *S,
                                      RcStats &rs) {
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    ++rs.rc;
    if (b.force_recheck && cls != 2 && cls != res) ++rs.viol;
    // The atomic on the canonical bit decides: an edge another test already removed stays
    // removed and keeps that test's SepSet.
    if (res && take_edge(P.adj, P.W, lo, hi)) {
        ++rs.rm;
        write_record(P, lo, hi, l, S);
    }
}

// FP64 decision of the Gram block G by one wavefront (all lanes get it): the register elimination,
// or, when M2 is numerically singular, the pseudo-inverse route on lane 0 with scratch `work`.
template <int KMAX>
__device__ inline int decide_wave(const double *G, int ld, int l, double tau, double *work, int mm, int lane) {
    int res = decide_elim<KMAX>(G, ld, l + 2, tau, lane);
    if (res < 0) {
        if (lane == 0) res = decide_gram64(G, ld, l, tau, work, mm);
        res = __shfl(res, 0, 64);
    }
    return res;
}

// Pairwise dot products of up to four FP64 standardized rows v[0..K) (levels 1 and 2, where the
// 16 x 16 MFMA tile would be mostly zero rows): each lane takes two consecutive samples of every
// block of 128 starting at x_first (blocks x_step apart) and returns its partial sums of the pairs
// (0,1), (0,2), (1,2), (0,3), (1,3), (2,3) in s.
__device__ inline void gram_small_part(const Prob &P, const int *v, int K, int lane, int64_t x_first, int64_t x_step,
                                       double (&s)[6]) {
    const int64_t mp = P.mp;
    const double *z0 = P.zt64 + (int64_t)v[0] * mp, *z1 = P.zt64 + (int64_t)v[1] * mp;
    const double *z2 = P.zt64 + (int64_t)v[K > 2 ? 2 : 0] * mp, *z3 = P.zt64 + (int64_t)v[K > 3 ? 3 : 0] * mp;
#pragma unroll
    for (int q = 0; q < 6; ++q) s[q] = 0.0;
    // mp is a multiple of 64, so both samples of a lane are inside whenever the first is.
#pragma unroll 2
    for (int64_t x = x_first + 2 * lane; x < mp; x += x_step) {
        const double2 a = *reinterpret_cast<const double2 *>(z0 + x);
        const double2 c = *reinterpret_cast<const double2 *>(z1 + x);
        const double2 e = K > 2 ? *reinterpret_cast<const double2 *>(z2 + x) : double2{0.0, 0.0};
        const double2 g = K > 3 ? *reinterpret_cast<const double2 *>(z3 + x) : double2{0.0, 0.0};
        s[0] = fma(a.y, c.y, fma(a.x, c.x, s[0]));
        s[1] = fma(a.y, e.y, fma(a.x, e.x, s[1]));
        s[2] = fma(c.y, e.y, fma(c.x, e.x, s[2]));
        s[3] = fma(a.y, g.y, fma(a.x, g.x, s[3]));
        s[4] = fma(c.y, g.y, fma(c.x, g.x, s[4]));
        s[5] = fma(e.y, g.y, fma(e.x, g.x, s[5]));
    }
}

// Writes the K x K Gram block (row stride 16, unit diagonal) from the pair sums of gram_small_part.
__device__ inline void gram_small_store(const double (&s)[6], int K, double *G) {
    const int pa[6] = {0, 0, 1, 0, 1, 2}, pb[6] = {1, 2, 2, 3, 3, 3};
    for (int r = 0; r < K; ++r) G[r * 16 + r] = 1.0;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        if (pb[q] < K) {
            G[pa[q] * 16 + pb[q]] = s[q];
            G[pb[q] * 16 + pa[q]] = s[q];
        }
}

// ---------------------------------------------------------------------------------------------
// Address-space-typed pointers
// ---------------------------------------------------------------------------------------------
// Accessors that pick LDS or global memory at run time would otherwise be merged by the compiler
// into one flat load (which waits on both memory counters); typed pointers keep ds_* and global_*
// instructions apart.
template <typename T> using lds_ptr = __attribute__((address_space(3))) T *;
template <typename T> using glb_ptr = __attribute__((address_space(1))) T *;

template <int V>
struct IntTag {
    static constexpr int value = V;
};

__device__ inline void lds_and(lds_ptr<unsigned long long> p, unsigned long long v) {
    __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
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

// The same table staged in LDS for one row: C(a, b) for a <= d, b <= L, row stride `cols`. An
// unranking is a chain of dependent table reads, so each read costs LDS latency instead of L2's.
struct LdsBinom {
    lds_ptr<const unsigned long long> t;
    int cols;
    __device__ unsigned long long operator()(int a, int b) const {
        if (b < 0 || a < b) return 0ull;
        return t[a * cols + b];
    }
};

template <typename T>
__host__ __device__ constexpr size_t lds_fixed_bytes() {
    return (sizeof(int) * kDcap + 15) / 16 * 16 + (sizeof(T) * kDcap + 15) / 16 * 16 +
           sizeof(unsigned long long) * kWcap;
}

// Wavefronts per SIMD the register allocation of k_level<T, L> is held to. A level there is a few
// rounds of work items of similar latency across all resident work-groups, so one more resident
// work-group per CU shortens it: FP32 levels 3 and 4 (129-139 registers otherwise) get four, and 6
// and 7 (162-183) three, at up to 4 spilled registers; levels 5 and 8 would spill 9-10 and are
// slower held to the next step.
template <typename T, int L>
constexpr int level_waves_per_simd() {
    if (sizeof(T) != 4) return 1;
    return (L == 3 || L == 4) ? 4 : ((L == 6 || L == 7) ? 3 : 1);
}

template <typename T, int L>
__global__ __launch_bounds__(kLevelThreads, (level_waves_per_simd<T, L>())) void k_level(Batch b, int R, int lds_bytes) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ long long s_grow, s_item;
    __shared__ int s_mode;  // bit 0: nb/ci in LDS, bit 1: C[N_i,N_i] in LDS, bit 2: live bits in LDS
    __shared__ int s_binoff;  // byte offset of the row's binomials in the dynamic LDS, or -1
    __shared__ long long s_tests, s_removed;
    // Removals found while testing are staged here and settled at the end of the item, so a
    // wavefront never waits on a device-scope atomic inside the test loop.
    __shared__ int s_nstage, s_nwin;
    __shared__ int s_stage_j[kStageCap];
    __shared__ unsigned long long s_stage_t[kStageCap];
    __shared__ unsigned long long s_rec_base;
    __shared__ int s_livepos[kDcap];   // positions p whose edge (i, N_i[p]) is live at item start
    __shared__ int s_perm[L == 1 ? kLevelThreads : 1];   // level 1: list positions of the item's ranks
    __shared__ long long s_scan[kLevelThreads / 64];

    DevState *st = b.st;
    const int done = st->done;
    const unsigned long long total = st->total_items, stride = st->item_stride;
    if (done) return;
    const int tid = threadIdx.x;
    // Typed LDS pointers: every access below compiles to a ds_* instruction, never a flat one.
    const lds_ptr<int> lds_nb = (lds_ptr<int>)(smem);
    const lds_ptr<T> lds_ci = (lds_ptr<T>)(smem + (sizeof(int) * kDcap + 15) / 16 * 16);
    const lds_ptr<unsigned long long> lds_live = (lds_ptr<unsigned long long>)(
        smem + (sizeof(int) * kDcap + 15) / 16 * 16 + (sizeof(T) * kDcap + 15) / 16 * 16);
    const lds_ptr<T> lds_blk = (lds_ptr<T>)(smem + lds_fixed_bytes<T>());
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
            // The first item of a work-group is its own index; later ones come from the queue
            // (which has none when every item had a work-group of its own).
            unsigned long long g = blockIdx.x;
            if (!first) {
                if (total <= gridDim.x) g = total;
                else if (tid == 0) g = gridDim.x + atomicAdd(&st->next_item, 1ull);
            }
            g = __shfl(g, 0, 64);
            // A re-check queue overflow stops the level (it is redone in FP64): no further items.
            if (__hip_atomic_load(&st->rq_overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) g = total;
            if (g >= total) {
                if (tid == 0) s_grow = -1;
            } else {
                // (in queue order, rows only grow: the search starts at the last row)
                long long lo = last_row, hi = b.total_rows;
                if (stride > 1ull) {
                    g = g * stride % total;
                    lo = 0;
                }
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
                    s_item = (long long)(g - (unsigned long long)b.item_off[lo]);
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
            if (tid == 0 && stats_pd >= 0) flush_stats<L>(b, b.probs[stats_pd], s_tests, s_removed);
            stats_pd = pd;
        }
        const Prob &P = b.probs[pd];
        const int64_t n = P.n, W = P.W;
        const int row = (int)(grow - b.row_base[pd]);
        const glb_ptr<const T> C = (glb_ptr<const T>)(P.C);
        unsigned long long *adj_row = P.adj + (int64_t)row * W;
        // Live bits of row i, refreshed at every item (other rows remove edges meanwhile); the load
        // is issued here so that it overlaps the staging below (one word per thread).
        static_assert(kWcap <= kLevelThreads, "one live-bit word per thread");
        unsigned long long live_w = 0ull;
        if (W <= kWcap && tid < W) live_w = live_word(adj_row + tid);
        if (grow != staged) {
            // The staging is a chain of dependent loads (degree, neighbour ids, then the entries of
            // C at those ids); loads that do not depend on each other are issued together: the
            // thread's first neighbour id with the binomials, and C[i, N_i] with the block
            // C[N_i, N_i] when the block is staged.
            d = __builtin_amdgcn_readfirstlane(P.deg[row]);
            const bool nb_lds = d <= kDcap;
            const bool blk_lds = nb_lds && (long long)d * d <= blk_cap;
            const int k_first = nb_lds && tid < d ? P.nbr[(int64_t)row * n + tid] : 0;
            if constexpr (L >= 2) {
                // The binomials this row's unranking reads, after the block when they fit.
                const long long off = (long long)lds_fixed_bytes<T>() +
                                      (blk_lds ? ((long long)d * d * (long long)sizeof(T) + 7) / 8 * 8 : 0);
                const int nbin = (d + 1) * (L + 1);
                const bool bin_lds = nb_lds && off + 8ll * nbin <= (long long)lds_bytes;
                if (bin_lds) {
                    const lds_ptr<unsigned long long> lb = (lds_ptr<unsigned long long>)(smem + off);
                    for (int e = tid; e < nbin; e += kLevelThreads) lb[e] = binom(e / (L + 1), e % (L + 1));
                }
                if (tid == 0) s_binoff = bin_lds ? (int)off : -1;
            }
            if (nb_lds)
                for (int p = tid; p < d; p += kLevelThreads) {
                    const int k = p == tid ? k_first : P.nbr[(int64_t)row * n + p];
                    lds_nb[p] = k;
                    if (!blk_lds) lds_ci[p] = C[(int64_t)row * n + k];
                }
            __syncthreads();
            if (blk_lds) {
                // C[N_i, N_i], then C[i, N_i]: each thread issues 8 independent gathers before
                // storing any.
                const int dd = d * d, de = dd + d;
                for (int e0 = tid; e0 < de; e0 += 8 * kLevelThreads) {
                    T v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int e = e0 + u * kLevelThreads;
                        v[u] = (T)0;
                        if (e < dd) {
                            const int p = e / d, q = e - p * d;
                            v[u] = C[(int64_t)lds_nb[p] * n + lds_nb[q]];
                        } else if (e < de) {
                            v[u] = C[(int64_t)row * n + lds_nb[e - dd]];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int e = e0 + u * kLevelThreads;
                        if (e < dd) lds_blk[e] = v[u];
                        else if (e < de) lds_ci[e - dd] = v[u];
                    }
                }
            }
            if (tid == 0) s_mode = (nb_lds ? 1 : 0) | (blk_lds ? 2 : 0) | (W <= kWcap ? 4 : 0);
            staged = grow;
        }
        if (W <= kWcap && tid < W) lds_live[tid] = live_w;
        __syncthreads();
        const int mode = __builtin_amdgcn_readfirstlane(s_mode);
        const glb_ptr<const int> nbg = (glb_ptr<const int>)(P.nbr + (int64_t)row * n);
        // When the neighbour list and live bits sit in LDS, the j loops run over the positions whose
        // edge is still live at item start (edges removed earlier cannot be tested), in order.
        int nlive = d;
        if ((mode & 5) == 5) {
            int base = 0;
            for (int p0 = 0; p0 < d; p0 += kLevelThreads) {
                const int p = p0 + tid;
                bool f = false;
                if (p < d) {
                    const int j = lds_nb[p];
                    f = (lds_live[j >> 6] >> (j & 63)) & 1ull;
                }
                long long tot = 0;
                const long long pre = block_exclusive_scan<kLevelThreads>(f ? 1 : 0, s_scan, tot);
                if (f) s_livepos[base + (int)pre] = p;
                base += (int)tot;
                __syncthreads();
            }
            nlive = base;
        }
        // A row longer than kDcap keeps its neighbour list in global memory. When its still-live
        // candidates fit, they are compacted into the LDS list itself (ids and C_ij, ascending j),
        // straight from the live bits: every live edge of G is an edge of the snapshot G'. Sets
        // are still ranked over the whole list (their ids and C_ik come from global memory). Level 1
        // only: long rows at higher levels are rare, and the extra placement costs the deeper
        // kernels a wavefront of occupancy in registers.
        bool compact = false;
        if (L == 1 && !(mode & 1) && (mode & 4)) {
            static_assert(kWcap <= kLevelThreads, "one live-bit word per thread");
            unsigned long long wv = 0ull;
            if (tid < W) {
                wv = lds_live[tid];
                // a caller-supplied G may carry stray bits: the diagonal and columns >= n
                if (tid == (row >> 6)) wv &= ~(1ull << (row & 63));
                if (tid == W - 1 && (n & 63)) wv &= (1ull << (n & 63)) - 1ull;
            }
            long long tot = 0;
            const long long pre = block_exclusive_scan<kLevelThreads>((long long)__popcll(wv), s_scan, tot);
            if (tot <= kDcap) {
                int q = (int)pre;
                while (wv) {
                    const int j = tid * 64 + __ffsll((long long)wv) - 1;
                    lds_nb[q] = j;
                    lds_ci[q] = C[(int64_t)row * n + j];
                    ++q;
                    wv &= wv - 1ull;
                }
                nlive = (int)tot;
                compact = true;
            }
            __syncthreads();
        }
        const double tau = P.tau[L];
        const float tl = P.t[L], band = P.band[L];

        const unsigned long long nS = binom(d, L);
        unsigned long long wlo, whi;
        rank_window(b, nS, wlo, whi);
        const long long Rr = item_sets(d, L, R, b.lane_tests);
        const long long r0 = (long long)wlo + s_item * Rr;
        const long long r1 = (long long)whi < r0 + Rr ? (long long)whi : r0 + Rr;
        const long long nr = r1 - r0;
        // `split` threads share each conditioning set and divide its j loop; each group of them
        // takes qn sets. At levels 1 and 2 a set needs no factor or a 2 x 2 one, so up to a whole
        // wavefront shares it: its lanes then read rows of C (or of the staged block) at
        // consecutive neighbour positions, instead of 64 rows at once, and a group's later sets skip
        // the edges its earlier ones removed (at level 2 that cuts the tests run by a fifth). Above
        // (where a set's factor costs more than its j loop), one thread per set, unless the item has
        // fewer sets than threads.
        int split = 1;
        if (L <= kWaveSetLevels) {
            // A set's lanes are sized to the live list: when few edges of the row are still live
            // (a row left with its surviving edges, which every set must test), a wavefront takes
            // several sets at once, and its lanes still carry about kBatch candidates each.
            split = 64;
            if ((mode & 5) == 5 || compact)
                while (split > b.set_lanes && (split / 2) * 8 >= nlive) split >>= 1;
        } else if (nr < kLevelThreads) {
            while (split * 2 * nr <= kLevelThreads) split *= 2;
        }
        const int groups = kLevelThreads / split;
        const int slice = tid % split;
        const int qn = (int)((nr + groups - 1) / groups);
        // Level 1: the wavefronts of an item take its sets round robin, so that all of them start
        // with the item's first sets (the strongest, when the order sorted them). Above: each
        // thread group takes qn consecutive sets and steps through them by the successor rule.
        const bool interleave = L == 1;
        const long long my_t = interleave ? r0 + tid / split : r0 + (long long)(tid / split) * qn;
        const long long my_end = interleave ? r1 : (my_t + qn < r1 ? my_t + qn : r1);
        const long long t_stride = interleave ? groups : 1;
        // Level 1 after a sorted shared-set order: rank t is list position perm[t]; the item's
        // positions are staged in LDS first (an item has at most kLevelThreads ranks at level 1),
        // so the set loop does not wait on a global load per set.
        const bool perm = L == 1 && l1_perm_row(b, d, W, n);
        const bool perm_lds = perm && nr <= kLevelThreads;   // (more ranks per item: read in place)
        const glb_ptr<const int> permg = (glb_ptr<const int>)(P.nbr + (int64_t)row * n + d);
        if constexpr (L == 1) {
            if (perm_lds) {
                if (tid < nr) s_perm[tid] = permg[r0 + tid];
                __syncthreads();
            }
        }
        int since_refresh = 0;

        int binoff = -1;
        if constexpr (L >= 2) binoff = __builtin_amdgcn_readfirstlane(s_binoff);
        const LdsBinom lbinom{(lds_ptr<const unsigned long long>)(smem + (binoff > 0 ? binoff : 0)), L + 1};
        int P_[L];
#pragma unroll
        for (int c = 0; c < L; ++c) P_[c] = 0;
        if (my_t < my_end && L > 1) {
            if (binoff > 0) comb_unrank<L>(d, (unsigned long long)my_t, P_, lbinom);
            else comb_unrank<L>(d, (unsigned long long)my_t, P_, binom);
        }
        // The set loop, specialised on where the row's data sits: K = 7 all of it in LDS, K = 5 all
        // but the block C[N_i, N_i] (gathered from global C), K = 1 a row longer than kDcap whose
        // live candidates were compacted into LDS, K = 0 any mix (decided per access). In the
        // specialised forms every load of a set is branch-free, so the compiler issues them
        // together instead of waiting on each one.
        auto run_sets = [&](auto kind) {
            constexpr int K = decltype(kind)::value;
            // Candidates: list positions of the live list (K = 5, 7), entries of the compacted
            // list (K = 1), or all positions of N_i (K = 0).
            const int ncand = K != 0 ? nlive : d;
            const int psteps = (ncand + split - 1) / split;
            auto POS = [&](int idx) -> int {
                if constexpr (K >= 5) return s_livepos[idx];
                else return idx;
            };
            // Id, C_ik and C[N_p, N_q] at positions of N_i (sets always; candidates unless K = 1).
            auto NB = [&](int p) -> int {
                if constexpr (K >= 5) return lds_nb[p];
                else if constexpr (K == 1) return nbg[p];
                else return (mode & 1) ? lds_nb[p] : nbg[p];
            };
            auto CI = [&](int p) -> T {
                if constexpr (K >= 5) return lds_ci[p];
                else if constexpr (K == 1) return C[(int64_t)row * n + nbg[p]];
                else return (mode & 1) ? lds_ci[p] : C[(int64_t)row * n + nbg[p]];
            };
            auto CS = [&](int p, int q) -> T {
                if constexpr (K == 7) return p == q ? (T)1 : lds_blk[p * d + q];
                // From global C, the row of the set element q (C is exactly symmetric): at level 1
                // the lanes of a wavefront share q and read ascending columns N_p of one row.
                else if constexpr (K == 5) return p == q ? (T)1 : C[(int64_t)lds_nb[q] * n + lds_nb[p]];
                else if constexpr (K == 1) return p == q ? (T)1 : C[(int64_t)nbg[q] * n + nbg[p]];
                else {
                    if (p == q) return (T)1;
                    return (mode & 2) ? lds_blk[p * d + q] : C[(int64_t)NB(q) * n + NB(p)];
                }
            };
            auto LIVE = [&](int j) -> bool {
                unsigned long long wv;
                if constexpr (K != 0) wv = lds_live[j >> 6];
                else wv = (mode & 4) ? lds_live[j >> 6] : live_word(adj_row + (j >> 6));
                return (wv >> (j & 63)) & 1ull;
            };
            for (int step = 0; step < qn; ++step) {
                const long long t = my_t + step * t_stride;
                if (t >= my_end) break;
                if constexpr (L == 1) P_[0] = perm_lds ? s_perm[t - r0] : (perm ? permg[t] : (int)t);
                else if (step > 0) comb_next<L>(d, P_);

                // Shared per-S work: Cholesky of M2 = C[S,S], y = L^-1 C[S,i]^T, H11 = 1 - y.y.
                SetFactor<T, L> f;
                f.build(P_, CS, CI);
                int sid[L];
    #pragma unroll
                for (int c = 0; c < L; ++c) sid[c] = NB(P_[c]);

                // Candidates j are taken kBatch at a time: their liveness and the values each test
                // reads (C[N_p, S] and C[i, N_p]) are all loaded before the first test of the batch.
                constexpr int kBatch = L == 1 ? 8 : (L <= 3 ? 4 : (L <= 7 ? 2 : 1));
                for (int pp0 = 0; pp0 < psteps; pp0 += kBatch) {
                    if ((K != 0 || (mode & 4)) && (since_refresh += kBatch) >= 16) {
                        // Fold in removals made by other work-groups since the row was staged.
                        since_refresh = 0;
                        const int idx = pp0 * split + slice;
                        if (idx < ncand) {
                            int j;
                            if constexpr (K == 1) j = lds_nb[idx];
                            else j = NB(POS(idx));
                            lds_and(lds_live + (j >> 6), live_word(adj_row + (j >> 6)));
                        }
                    }
                    T col[kBatch][L], cij[kBatch];
                    int jb[kBatch];
                    bool go[kBatch];
    #pragma unroll
                    for (int u = 0; u < kBatch; ++u) {
                        const int idx = (pp0 + u) * split + slice;
                        bool ok = pp0 + u < psteps && idx < ncand;
                        const int p = ok ? POS(idx) : 0;
                        int j;
                        if constexpr (K == 1) {
                            // compacted entry p: the candidate is excluded by id, not position
                            j = ok ? lds_nb[p] : 0;
    #pragma unroll
                            for (int c = 0; c < L; ++c) ok &= sid[c] != j;
                        } else {
    #pragma unroll
                            for (int c = 0; c < L; ++c) ok &= P_[c] != p;
                            j = ok ? NB(p) : 0;
                        }
                        ok = ok && LIVE(j);
                        go[u] = ok;
                        jb[u] = j;
                        if constexpr (K == 1) {
    #pragma unroll
                            for (int r = 0; r < L; ++r) col[u][r] = ok ? C[(int64_t)sid[r] * n + j] : (T)0;
                            cij[u] = ok ? lds_ci[p] : (T)0;
                        } else {
    #pragma unroll
                            for (int r = 0; r < L; ++r) col[u][r] = ok ? CS(p, P_[r]) : (T)0;
                            cij[u] = ok ? CI(p) : (T)0;
                        }
                    }
    #pragma unroll
                    for (int u = 0; u < kBatch; ++u) {
                        if (!go[u]) continue;
                        const int j = jb[u];
                        ++my_tests;
                        const int dec = f.test_vals(col[u], cij[u], tau, tl, band);
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
                                // the rank; at level 1 the list position itself (rank and
                                // position differ once the order sorted the sets)
                                s_stage_t[slot] = L == 1 ? (unsigned long long)P_[0] : (unsigned long long)t;
                            } else {
                                const int lo = row < j ? row : j, hi = row < j ? j : row;
                                if (take_edge(P.adj, W, lo, hi)) {
                                    ++my_removed;
                                    write_record(P, lo, hi, L, sid);
                                }
                            }
                            if (K != 0 || (mode & 4)) lds_and(lds_live + (j >> 6), ~(1ull << (j & 63)));
                        }
                    }
                }
            }
        };
        if (mode == 7) run_sets(IntTag<7>{});
        else if (mode == 5) run_sets(IntTag<5>{});
        else if (L == 1 && compact) run_sets(IntTag<L == 1 ? 1 : 0>{});
        else run_sets(IntTag<0>{});
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
                    if (binoff > 0) comb_unrank<L>(d, srank, Q, lbinom);
                    else comb_unrank<L>(d, srank, Q, binom);
                    int qs[L];
#pragma unroll
                    for (int c = 0; c < L; ++c) qs[c] = (mode & 1) ? lds_nb[Q[c]] : nbg[Q[c]];
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
    if (tid == 0 && stats_pd >= 0) flush_stats<L>(b, b.probs[stats_pd], s_tests, s_removed);
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
    const int done = st->done;
    const unsigned long long total = st->total_items, stride = st->item_stride;
    if (done) return;
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
            if (!first) {
                if (total <= gridDim.x) g = total;
                else if (tid == 0) g = gridDim.x + atomicAdd(&st->next_item, 1ull);
            }
            g = __shfl(g, 0, 64);
            // A re-check queue overflow stops the level (it is redone in FP64): no further items.
            if (__hip_atomic_load(&st->rq_overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) g = total;
            if (g >= total) {
                if (tid == 0) s_grow = -1;
            } else {
                long long lo = last_row, hi = b.total_rows;
                if (stride > 1ull) {
                    g = g * stride % total;
                    lo = 0;
                }
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
                    s_r0 = (long long)(g - (unsigned long long)b.item_off[lo]);
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
            if (tid == 0 && stats_pd >= 0) flush_stats<L>(b, b.probs[stats_pd], s_tests, s_removed);
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
        unsigned long long wlo, whi;
        rank_window(b, nS, wlo, whi);
        const long long r0 = (long long)wlo + s_r0 * R;
        const long long r1 = (long long)whi < r0 + R ? (long long)whi : r0 + R;
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
    if (tid == 0 && stats_pd >= 0) flush_stats<L>(b, b.probs[stats_pd], s_tests, s_removed);
}

template <typename T, int L>
inline hipError_t launch_level_t(hipStream_t s, const Batch &b, int R, int lds_bytes, int grid) {
    if constexpr (L <= kFastLevels)
        hipLaunchKernelGGL((k_level<T, L>), dim3(grid), dim3(kLevelThreads), lds_bytes, s, b, R, lds_bytes);
    else
        hipLaunchKernelGGL((k_level_deep<T, L>), dim3(grid), dim3(kLevelThreads), 0, s, b, R);
    return hipGetLastError();
}

// Launch and occupancy query of the level kernel of `level` among the instances L .. LMAX.
template <typename T, int L, int LMAX>
struct LevelRange {
    static hipError_t launch(hipStream_t s, const Batch &b, int level, int R, int lds, int grid) {
        if (level == L) return launch_level_t<T, L>(s, b, R, lds, grid);
        return LevelRange<T, L + 1, LMAX>::launch(s, b, level, R, lds, grid);
    }
    static int occupancy(int level, int lds_bytes) {
        if (level != L) return LevelRange<T, L + 1, LMAX>::occupancy(level, lds_bytes);
        int nb = 0;
        hipError_t e;
        if constexpr (L <= kFastLevels)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_level<T, L>, kLevelThreads, lds_bytes);
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_level_deep<T, L>, kLevelThreads, 0);
        return e == hipSuccess ? nb : 0;
    }
};
template <typename T, int LMAX>
struct LevelRange<T, LMAX + 1, LMAX> {
    static hipError_t launch(hipStream_t, const Batch &, int, int, int, int) { return hipErrorInvalidValue; }
    static int occupancy(int, int) { return 0; }
};

// Entry points of the instantiating units (levels 1 .. kFastLevels, or the deep levels above).
hipError_t launch_level_fast_f32(hipStream_t s, const Batch &b, int level, int R, int lds, int grid);
hipError_t launch_level_fast_f64(hipStream_t s, const Batch &b, int level, int R, int lds, int grid);
hipError_t launch_level_deep(hipStream_t s, const Batch &b, int level, int R, int lds, int grid);
int occupancy_level_fast_f32(int level, int lds_bytes);
int occupancy_level_fast_f64(int level, int lds_bytes);
int occupancy_level_deep(int prec, int level);

}  // namespace pcg
