// Orientation of the skeleton into a CPDAG: the step of the PC algorithm that follows the skeleton
// (Sec. 2.4 names it; the paper keeps it on the CPU). Unshielded colliders come from the SepSets,
// then the propagation rules of Meek (1995) R1-R3 run in synchronous rounds.
//
// State, as bit matrices of n rows x W words:
//   OUT[x] bit y: the edge x - y has an arrowhead at y (the caller's output);
//   IN[x]  bit y: the edge x - y has an arrowhead at x (the transpose of OUT).
// With A = the skeleton: x -> y iff OUT[x]_y & !IN[x]_y; x - y undirected iff A[x]_y & !OUT[x]_y &
// !IN[x]_y; both arrowheads make a bidirected edge (two colliders disagreeing), which no rule uses.
//
// Conventions (independent of the order of work, so the result is unique):
//   * every unshielded triple i - k - j is judged on the skeleton and SepSets alone;
//   * a round proposes x -> y for every undirected x - y that R1, R2 or R3 orients in the state at
//     the start of the round, and applies the proposals together; an edge proposed both ways in
//     the same round stays undirected.
#include "pc_dev.h"

namespace pcg {

constexpr int kOrientThreads = 256;

__device__ inline bool bit_of(const unsigned long long *row, int64_t j) { return (row[j >> 6] >> (j & 63)) & 1ull; }

__global__ __launch_bounds__(kOrientThreads) void k_orient_clear(unsigned long long *a, int64_t words, int *sep_idx,
                                                                 int64_t pairs, int *flag) {
    const int64_t t = (int64_t)blockIdx.x * kOrientThreads + threadIdx.x, stride = (int64_t)gridDim.x * kOrientThreads;
    for (int64_t e = t; e < words; e += stride) a[e] = 0ull;
    for (int64_t e = t; e < pairs; e += stride) sep_idx[e] = -1;
    if (t == 0) *flag = 0;
}

// sep_idx[i * n + j] (i < j) = index of the SepSet record of the pair; -1: removed at level 0
// (empty SepSet). Records with ids or levels out of range are ignored.
__global__ __launch_bounds__(kOrientThreads) void k_sep_index(const pc_sep_rec *recs, int64_t nrec, int64_t n,
                                                              int *sep_idx) {
    const int64_t r = (int64_t)blockIdx.x * kOrientThreads + threadIdx.x;
    if (r >= nrec) return;
    const pc_sep_rec &e = recs[r];
    if (e.i < 0 || e.j < 0 || e.i >= n || e.j >= n || e.i == e.j || e.level < 1 || e.level > PC_MAX_LEVEL) return;
    const int64_t lo = e.i < e.j ? e.i : e.j, hi = e.i < e.j ? e.j : e.i;
    sep_idx[lo * n + hi] = (int)r;
}

// One work-group per node k: every neighbour a of k against the neighbours b > a of k that are not
// adjacent to a (word-parallel on the bit rows); k outside SepSet(a, b) makes a -> k <- b.
__global__ __launch_bounds__(kOrientThreads) void k_vstruct(const unsigned long long *A, int64_t n, int64_t W,
                                                            const pc_sep_rec *recs, const int *sep_idx,
                                                            unsigned long long *OUT, unsigned long long *IN) {
    const int64_t k = blockIdx.x;
    const unsigned long long *ak = A + k * W;
    for (int64_t a = threadIdx.x; a < n; a += kOrientThreads) {
        if (a == k || !bit_of(ak, a)) continue;
        const unsigned long long *aa = A + a * W;
        for (int64_t w = a >> 6; w < W; ++w) {
            unsigned long long cand = ak[w] & ~aa[w];
            if (w == (a >> 6)) cand &= (a & 63) == 63 ? 0ull : ~((2ull << (a & 63)) - 1ull);   // b > a
            while (cand) {
                const int64_t b = w * 64 + (__ffsll((long long)cand) - 1);
                cand &= cand - 1;
                if (b == k || b >= n) continue;
                const int r = sep_idx[a * n + b];
                bool in_s = false;
                if (r >= 0) {
                    const pc_sep_rec &e = recs[r];
                    for (int c = 0; c < e.level; ++c) in_s |= e.S[c] == (int)k;
                }
                if (!in_s) {
                    atomicOr(IN + k * W + (a >> 6), 1ull << (a & 63));
                    atomicOr(IN + k * W + (b >> 6), 1ull << (b & 63));
                    atomicOr(OUT + a * W + (k >> 6), 1ull << (k & 63));
                    atomicOr(OUT + b * W + (k >> 6), 1ull << (k & 63));
                }
            }
        }
    }
}

// Proposals of one round: work-group per x, threads over its undirected neighbours y.
__global__ __launch_bounds__(kOrientThreads) void k_meek_propose(const unsigned long long *A, int64_t n, int64_t W,
                                                                 const unsigned long long *OUT,
                                                                 const unsigned long long *IN,
                                                                 unsigned long long *P) {
    const int64_t x = blockIdx.x;
    const unsigned long long *ax = A + x * W, *ox = OUT + x * W, *ix = IN + x * W;
    for (int64_t y = threadIdx.x; y < n; y += kOrientThreads) {
        if (y == x || !bit_of(ax, y) || bit_of(ox, y) || bit_of(ix, y)) continue;   // undirected x - y
        const unsigned long long *ay = A + y * W, *oy = OUT + y * W, *iy = IN + y * W;
        bool r = false;
        for (int64_t w = 0; w < W && !r; ++w) {
            const unsigned long long into_x = ix[w] & ~ox[w];    // a -> x
            const unsigned long long from_x = ox[w] & ~ix[w];    // x -> a
            const unsigned long long into_y = iy[w] & ~oy[w];    // a -> y
            r = (into_x & ~ay[w]) != 0ull                        // R1 (a != y: y - x is undirected)
                || (from_x & into_y) != 0ull;                    // R2
        }
        if (!r) {
            // R3: two non-adjacent c, d with x - c, x - d undirected and c -> y, d -> y
            for (int64_t w = 0; w < W && !r; ++w) {
                unsigned long long cs = ax[w] & ~ix[w] & ~ox[w] & iy[w] & ~oy[w];
                while (cs && !r) {
                    const int64_t c = w * 64 + (__ffsll((long long)cs) - 1);
                    cs &= cs - 1;
                    if (c >= n) break;   // stray bits past column n - 1 of a caller's matrix
                    const unsigned long long *ac = A + c * W;
                    for (int64_t v = 0; v < W && !r; ++v) {
                        unsigned long long ds = ax[v] & ~ix[v] & ~ox[v] & iy[v] & ~oy[v] & ~ac[v];
                        if (v == (c >> 6)) ds &= ~(1ull << (c & 63));
                        r = ds != 0ull;
                    }
                }
            }
        }
        if (r) atomicOr(P + x * W + (y >> 6), 1ull << (y & 63));
    }
}

// Applies the proposals of P that are not opposed (P[y] bit x), counts them in *flag, and clears
// the other proposal buffer Q for the next round.
__global__ __launch_bounds__(kOrientThreads) void k_meek_apply(int64_t n, int64_t W, const unsigned long long *P,
                                                               unsigned long long *Q, unsigned long long *OUT,
                                                               unsigned long long *IN, int *flag) {
    const int64_t t = (int64_t)blockIdx.x * kOrientThreads + threadIdx.x;
    if (t >= n * W) return;
    Q[t] = 0ull;
    const int64_t x = t / W, w = t - x * W;
    unsigned long long p = P[t];
    int changed = 0;
    while (p) {
        const int64_t y = w * 64 + (__ffsll((long long)p) - 1);
        p &= p - 1;
        if (bit_of(P + y * W, x)) continue;   // proposed both ways: stays undirected
        atomicOr(OUT + x * W + w, 1ull << (y & 63));
        atomicOr(IN + y * W + (x >> 6), 1ull << (x & 63));
        ++changed;
    }
    if (changed) atomicAdd(flag, changed);
}

__global__ void k_flag_reset(int *flag) { *flag = 0; }

hipError_t launch_orient_setup(hipStream_t s, int64_t n, const unsigned long long *A, const pc_sep_rec *recs,
                               int64_t nrec, unsigned long long *OUT, unsigned long long *IN,
                               unsigned long long *P0, unsigned long long *P1, int *sep_idx, int *flag) {
    const int64_t W = (n + 63) / 64, words = n * W;
    const int64_t blocks = (n * n + kOrientThreads - 1) / kOrientThreads;
    const unsigned grid = (unsigned)(blocks < 4096 ? blocks : 4096);
    hipLaunchKernelGGL(k_orient_clear, dim3(grid), dim3(kOrientThreads), 0, s, OUT, words, sep_idx, n * n, flag);
    hipLaunchKernelGGL(k_orient_clear, dim3(grid), dim3(kOrientThreads), 0, s, IN, words, sep_idx, 0, flag);
    hipLaunchKernelGGL(k_orient_clear, dim3(grid), dim3(kOrientThreads), 0, s, P0, words, sep_idx, 0, flag);
    hipLaunchKernelGGL(k_orient_clear, dim3(grid), dim3(kOrientThreads), 0, s, P1, words, sep_idx, 0, flag);
    if (nrec > 0)
        hipLaunchKernelGGL(k_sep_index, dim3((unsigned)((nrec + kOrientThreads - 1) / kOrientThreads)),
                           dim3(kOrientThreads), 0, s, recs, nrec, n, sep_idx);
    hipLaunchKernelGGL(k_vstruct, dim3((unsigned)n), dim3(kOrientThreads), 0, s, A, n, W, recs, sep_idx, OUT, IN);
    return hipGetLastError();
}

hipError_t launch_orient_round(hipStream_t s, int64_t n, const unsigned long long *A, unsigned long long *OUT,
                               unsigned long long *IN, unsigned long long *P, unsigned long long *Q, int *flag) {
    const int64_t W = (n + 63) / 64;
    hipLaunchKernelGGL(k_flag_reset, dim3(1), dim3(1), 0, s, flag);
    hipLaunchKernelGGL(k_meek_propose, dim3((unsigned)n), dim3(kOrientThreads), 0, s, A, n, W, OUT, IN, P);
    hipLaunchKernelGGL(k_meek_apply, dim3((unsigned)((n * W + kOrientThreads - 1) / kOrientThreads)),
                       dim3(kOrientThreads), 0, s, n, W, P, Q, OUT, IN, flag);
    return hipGetLastError();
}

}  // namespace pcg
