// Correlation matrix C = Z^T Z on MFMA, with the level-0 CI test fused into the epilogue.
//
// Level 0 (Sec. 3.2, Algorithm 3) tests every pair i < j with S = {} and, as Sec. 4.3 notes,
// reduces to comparing the Fisher z of C[V_i,V_j] with tau_0 (Eq. 5-6). Here that test runs on the
// 64 x 64 output tile while it is still in registers, and the tile's adjacency bits are packed
// into the bit matrix, so no separate level-0 kernel or n x n adjacency pass exists.
//
// Only upper-triangle tiles are launched (C is symmetric); each writes its tile and the mirror.
// One launch serves a whole batch: blocks map to (problem, tile) through the tile offsets.
// Precision paths:
//   FP64   : v_mfma_f64_16x16x4f64, exact FP64 decision |atanh(c)| <= tau_0.
//   FP32   : v_mfma_f32_16x16x4f32 on the FP32 copy of Z.
//   BF16x3 : v_mfma_f32_16x16x32_bf16 on hi*hi + hi*lo + lo*hi, FP32 accumulation.
// On the two low-precision paths a pair whose |c| lies within eps_c of tanh(tau_0) is re-done in
// FP64 as a dot product of the FP64 standardized columns, so every level-0 decision equals the
// FP64 one.
#include "pc_dev.h"

namespace pcg {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Fisher z of Eq. 5; +inf for |r| >= 1.
__device__ inline double fisher_z(double r) {
    if (!(fabs(r) < 1.0)) return INFINITY;
    return fabs(0.5 * log((1.0 + r) / (1.0 - r)));
}

template <int PREC> struct Tr;
template <> struct Tr<PC_PREC_FP32> {
    using T = float;
    using acc_t = floatx4;
    static constexpr int BK = 16;
};
template <> struct Tr<PC_PREC_FP64> {
    using T = double;
    using acc_t = doublex4;
    static constexpr int BK = 16;
};
template <> struct Tr<PC_PREC_BF16X3> {
    using T = float;
    using acc_t = floatx4;
    static constexpr int BK = 32;
};

constexpr int kT = 64;  // output tile edge

template <int PREC>
struct Smem;
template <> struct Smem<PC_PREC_FP32> {
    float A[16][kT + 4];
    float B[16][kT + 4];
};
template <> struct Smem<PC_PREC_FP64> {
    double A[16][kT + 2];
    double B[16][kT + 2];
};
template <> struct Smem<PC_PREC_BF16X3> {
    uint16_t Ahi[kT][40], Alo[kT][40], Bhi[kT][40], Blo[kT][40];
};

// Operands of one problem, copied to registers once (a Prob lives in global memory, and every
// barrier would otherwise force its fields to be reloaded).
struct Operands {
    int64_t n, mp;
    const double *zt64;
    const void *zlo, *zhi;
};

// One thread's share of the next K block of both operand tiles, held in registers between the
// global loads and the LDS stores so the loads can overlap the previous block's products.
template <int PREC> struct Frag;
template <> struct Frag<PC_PREC_FP32> { float4 a, b; };
template <> struct Frag<PC_PREC_FP64> { double2 a0, a1, b0, b1; };
template <> struct Frag<PC_PREC_BF16X3> { uint4 ah, al, bh, bl; };

template <int PREC>
__device__ inline void fetch_tiles(Frag<PREC> &f, const Operands &a, int64_t a0, int64_t b0, int64_t k0, int tid) {
    const int row = tid >> 2;
    if constexpr (PREC == PC_PREC_FP32) {
        const int kq = (tid & 3) * 4;
        const float *z = static_cast<const float *>(a.zlo);
        f.a = make_float4(0.f, 0.f, 0.f, 0.f);
        f.b = f.a;
        if (a0 + row < a.n) f.a = *reinterpret_cast<const float4 *>(z + (a0 + row) * a.mp + k0 + kq);
        if (b0 + row < a.n) f.b = *reinterpret_cast<const float4 *>(z + (b0 + row) * a.mp + k0 + kq);
    } else if constexpr (PREC == PC_PREC_FP64) {
        const int kq = (tid & 3) * 4;
        const double *z = a.zt64;
        f.a0 = make_double2(0.0, 0.0);
        f.a1 = f.b0 = f.b1 = f.a0;
        if (a0 + row < a.n) {
            const double2 *p = reinterpret_cast<const double2 *>(z + (a0 + row) * a.mp + k0 + kq);
            f.a0 = p[0];
            f.a1 = p[1];
        }
        if (b0 + row < a.n) {
            const double2 *p = reinterpret_cast<const double2 *>(z + (b0 + row) * a.mp + k0 + kq);
            f.b0 = p[0];
            f.b1 = p[1];
        }
    } else {
        const int k8 = (tid & 3) * 8;
        const uint16_t *zh = static_cast<const uint16_t *>(a.zhi);
        const uint16_t *zl = static_cast<const uint16_t *>(a.zlo);
        f.ah = make_uint4(0, 0, 0, 0);
        f.al = f.bh = f.bl = f.ah;
        if (a0 + row < a.n) {
            f.ah = *reinterpret_cast<const uint4 *>(zh + (a0 + row) * a.mp + k0 + k8);
            f.al = *reinterpret_cast<const uint4 *>(zl + (a0 + row) * a.mp + k0 + k8);
        }
        if (b0 + row < a.n) {
            f.bh = *reinterpret_cast<const uint4 *>(zh + (b0 + row) * a.mp + k0 + k8);
            f.bl = *reinterpret_cast<const uint4 *>(zl + (b0 + row) * a.mp + k0 + k8);
        }
    }
}

template <int PREC>
__device__ inline void stage_tiles(Smem<PREC> &sm, const Frag<PREC> &f, int tid) {
    const int row = tid >> 2;
    if constexpr (PREC == PC_PREC_FP32) {
        const int kq = (tid & 3) * 4;
        sm.A[kq + 0][row] = f.a.x; sm.A[kq + 1][row] = f.a.y;
        sm.A[kq + 2][row] = f.a.z; sm.A[kq + 3][row] = f.a.w;
        sm.B[kq + 0][row] = f.b.x; sm.B[kq + 1][row] = f.b.y;
        sm.B[kq + 2][row] = f.b.z; sm.B[kq + 3][row] = f.b.w;
    } else if constexpr (PREC == PC_PREC_FP64) {
        const int kq = (tid & 3) * 4;
        sm.A[kq + 0][row] = f.a0.x; sm.A[kq + 1][row] = f.a0.y;
        sm.A[kq + 2][row] = f.a1.x; sm.A[kq + 3][row] = f.a1.y;
        sm.B[kq + 0][row] = f.b0.x; sm.B[kq + 1][row] = f.b0.y;
        sm.B[kq + 2][row] = f.b1.x; sm.B[kq + 3][row] = f.b1.y;
    } else {
        const int k8 = (tid & 3) * 8;
        *reinterpret_cast<uint4 *>(&sm.Ahi[row][k8]) = f.ah;
        *reinterpret_cast<uint4 *>(&sm.Alo[row][k8]) = f.al;
        *reinterpret_cast<uint4 *>(&sm.Bhi[row][k8]) = f.bh;
        *reinterpret_cast<uint4 *>(&sm.Blo[row][k8]) = f.bl;
    }
}

template <int PREC>
__device__ inline void mma_step(const Smem<PREC> &sm, typename Tr<PREC>::acc_t (&acc)[2][2],
                                int lane, int wr, int wc) {
    const int li = lane & 15, lk = lane >> 4;
    if constexpr (PREC == PC_PREC_FP32) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            float af[2], bf[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                af[x] = sm.A[kk * 4 + lk][wr * 32 + x * 16 + li];
                bf[x] = sm.B[kk * 4 + lk][wc * 32 + x * 16 + li];
            }
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int nj = 0; nj < 2; ++nj)
                    acc[mi][nj] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mi], bf[nj], acc[mi][nj], 0, 0, 0);
        }
    } else if constexpr (PREC == PC_PREC_FP64) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            double af[2], bf[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                af[x] = sm.A[kk * 4 + lk][wr * 32 + x * 16 + li];
                bf[x] = sm.B[kk * 4 + lk][wc * 32 + x * 16 + li];
            }
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int nj = 0; nj < 2; ++nj)
                    acc[mi][nj] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[mi], bf[nj], acc[mi][nj], 0, 0, 0);
        }
    } else {
        bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            ah[x] = *reinterpret_cast<const bf16x8 *>(&sm.Ahi[wr * 32 + x * 16 + li][lk * 8]);
            al[x] = *reinterpret_cast<const bf16x8 *>(&sm.Alo[wr * 32 + x * 16 + li][lk * 8]);
            bh[x] = *reinterpret_cast<const bf16x8 *>(&sm.Bhi[wc * 32 + x * 16 + li][lk * 8]);
            bl[x] = *reinterpret_cast<const bf16x8 *>(&sm.Blo[wc * 32 + x * 16 + li][lk * 8]);
        }
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int nj = 0; nj < 2; ++nj) {
                acc[mi][nj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mi], bl[nj], acc[mi][nj], 0, 0, 0);
                acc[mi][nj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[mi], bh[nj], acc[mi][nj], 0, 0, 0);
                acc[mi][nj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mi], bh[nj], acc[mi][nj], 0, 0, 0);
            }
    }
}

// PF: K blocks staged per barrier. PF = 1 double-buffers single blocks (several work-groups per
// CU hide the load latency); PF > 1 stages 64 samples at a time, for launches with few tiles (or
// BF16x3), where one work-group per CU has to cover the latency by itself.
template <int PREC, int PF>
__global__ __launch_bounds__(256) void k_corr(Batch bt) {
    using T = typename Tr<PREC>::T;
    using acc_t = typename Tr<PREC>::acc_t;
    constexpr int BK = Tr<PREC>::BK;
    const int d = find_base(bt.tile_base, bt.count, blockIdx.x);
    const Prob &Pg = bt.probs[d];
    struct {
        int64_t n, m, mp, W;
        double *zt64;
        void *C;
        unsigned long long *adj;
        double t0, eps_c;
    } a = {Pg.n, Pg.m, Pg.mp, Pg.W, Pg.zt64, Pg.C, Pg.adj, Pg.t0, Pg.eps_c};
    const Operands ops = {Pg.n, Pg.mp, Pg.zt64, Pg.zlo, Pg.zhi};
    const double tau0 = Pg.tau[0];
    // Upper-triangle tile (ti <= tj) number k of this problem, rows of tiles taken in order.
    const int ntiles = (int)((a.n + kT - 1) / kT);
    int ti = 0, k = (int)(blockIdx.x - bt.tile_base[d]);
    while (k >= ntiles - ti) { k -= ntiles - ti; ++ti; }
    const int tj = ti + k;
    const int64_t a0 = (int64_t)ti * kT, b0 = (int64_t)tj * kT;
    const bool diag = ti == tj;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;

    constexpr int kPF = PF;
    static_assert(PF == 1 || PF * BK == 64, "groups of blocks span 64 samples");
    __shared__ Smem<PREC> sm[PF == 1 ? 2 : PF];
    __shared__ unsigned long long rowbits[kT], colbits[kT];
    __shared__ unsigned int blist[kT * kT];
    __shared__ int bcount;
    __shared__ int wg_removed, wg_rechecks;
    if (tid < kT) { rowbits[tid] = 0ull; colbits[tid] = 0ull; }
    if (tid == 0) { bcount = 0; wg_removed = 0; wg_rechecks = 0; }

    // FP32 / BF16x3: the MFMA accumulator holds one block of BK samples at a time (from zero),
    // and the blocks are added with compensated (two-sum) summation, so the rounding error of C
    // grows with the block length instead of with m.
    acc_t acc[2][2], sum[2][2], cmp[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[mi][nj][v] = sum[mi][nj][v] = cmp[mi][nj][v] = 0;

    auto compensate = [&]() {
        if constexpr (PREC != PC_PREC_FP64) {
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int nj = 0; nj < 2; ++nj)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const float x = acc[mi][nj][v], s0 = sum[mi][nj][v];
                        const float t = s0 + x, bp = t - s0;
                        cmp[mi][nj][v] += (s0 - (t - bp)) + (x - bp);
                        sum[mi][nj][v] = t;
                        acc[mi][nj][v] = 0.0f;
                    }
        }
    };
    if constexpr (PF == 1) {
        // Double buffer: block k + 1 is loaded and staged while block k is multiplied.
        Frag<PREC> frag;
        fetch_tiles<PREC>(frag, ops, a0, b0, 0, tid);
        stage_tiles<PREC>(sm[0], frag, tid);
        __syncthreads();
        int cur = 0;
        for (int64_t k0 = 0; k0 < a.mp; k0 += BK) {
            const bool more = k0 + BK < a.mp;
            if (more) fetch_tiles<PREC>(frag, ops, a0, b0, k0 + BK, tid);
            mma_step<PREC>(sm[cur], acc, lane, wr, wc);
            compensate();
            if (more) stage_tiles<PREC>(sm[cur ^ 1], frag, tid);
            __syncthreads();
            cur ^= 1;
        }
    } else {
        // mp is a multiple of 64, so every group of kPF blocks is whole.
        Frag<PREC> frag[kPF];
#pragma unroll
        for (int j = 0; j < kPF; ++j) fetch_tiles<PREC>(frag[j], ops, a0, b0, (int64_t)j * BK, tid);
#pragma unroll
        for (int j = 0; j < kPF; ++j) stage_tiles<PREC>(sm[j], frag[j], tid);
        __syncthreads();
        for (int64_t k0 = 0; k0 < a.mp; k0 += kPF * BK) {
            const bool more = k0 + kPF * BK < a.mp;
            if (more)
#pragma unroll
                for (int j = 0; j < kPF; ++j) fetch_tiles<PREC>(frag[j], ops, a0, b0, k0 + (int64_t)(kPF + j) * BK, tid);
#pragma unroll
            for (int j = 0; j < kPF; ++j) {
                mma_step<PREC>(sm[j], acc, lane, wr, wc);
                compensate();
            }
            __syncthreads();   // every wavefront is done with this group's LDS tiles
            if (more) {
#pragma unroll
                for (int j = 0; j < kPF; ++j) stage_tiles<PREC>(sm[j], frag[j], tid);
            }
            __syncthreads();
        }
    }
    if constexpr (PREC != PC_PREC_FP64) {
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int nj = 0; nj < 2; ++nj)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[mi][nj][v] = sum[mi][nj][v] + cmp[mi][nj][v];
    }

    // Epilogue: store C (tile and mirror), level-0 decisions, adjacency bits.
    T *C = static_cast<T *>(a.C);
    int removed = 0;
    const int li = lane & 15, lg = lane >> 4;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) {
            const int bl = wc * 32 + nj * 16 + li;
            const int64_t b = b0 + bl;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // Accumulator register v of lane (lg, li) holds row lg*4 + v of the 16 x 16 block
                // for the FP32/BF16 instructions and row lg + 4*v for v_mfma_f64_16x16x4f64.
                const int al = wr * 32 + mi * 16 + (PREC == PC_PREC_FP64 ? lg + 4 * v : lg * 4 + v);
                const int64_t ar = a0 + al;
                if (ar >= a.n || b >= a.n || ar > b) continue;  // a > b: written as the mirror
                if (ar == b) {
                    C[ar * a.n + b] = (T)1;
                    continue;
                }
                // Only (a < b) is stored from the accumulator; its mirror gets the same value, so C
                // is exactly symmetric (inside diagonal tiles (a,b) and (b,a) accumulate the BF16
                // cross terms in different orders).
                const T val = (T)acc[mi][nj][v];
                C[ar * a.n + b] = val;
                C[b * a.n + ar] = val;
                if (bt.corr_only) continue;   // C alone (an FP64 copy for a promoted level)
                bool keep, border = false;
                if constexpr (PREC == PC_PREC_FP64) {
                    keep = !(fisher_z((double)val) <= tau0);
                } else {
                    double x = fabs((double)val);
                    keep = x > a.t0 + a.eps_c;
                    border = !keep && x >= a.t0 - a.eps_c;
                    if (bt.force_recheck) border = true;
                }
                if (border) {
                    int k = atomicAdd(&bcount, 1);
                    blist[k] = ((unsigned)al << 8) | (unsigned)bl;
                } else if (keep) {
                    atomicOr(&rowbits[al], 1ull << bl);
                    atomicOr(&colbits[bl], 1ull << al);
                } else {
                    ++removed;
                }
            }
        }
    if (removed) atomicAdd(&wg_removed, removed);
    __syncthreads();

    if constexpr (PREC != PC_PREC_FP64) {
        // FP64 re-check of band pairs: one wave per pair, dot product of the FP64 columns.
        const int nb = bcount;
        for (int k = wave; k < nb; k += 4) {
            const unsigned e = blist[k];
            const int al = (int)(e >> 8), bl = (int)(e & 255u);
            const double *za = a.zt64 + (a0 + al) * a.mp;
            const double *zb = a.zt64 + (b0 + bl) * a.mp;
            double s = 0.0;
            for (int64_t r = lane; r < a.m; r += 64) s += za[r] * zb[r];
            s = wave_sum(s);
            if (lane == 0) {
                const bool keep = !(fisher_z(s) <= tau0);
                if (keep) {
                    atomicOr(&rowbits[al], 1ull << bl);
                    atomicOr(&colbits[bl], 1ull << al);
                } else {
                    atomicAdd(&wg_removed, 1);
                }
                atomicAdd(&wg_rechecks, 1);
            }
        }
        __syncthreads();
    }

    if (bt.corr_only) return;
    const int64_t W = a.W;
    if (tid < kT) {
        const int64_t r = a0 + tid;
        if (r < a.n) a.adj[r * W + tj] = rowbits[tid] | (diag ? colbits[tid] : 0ull);
    } else if (tid < 2 * kT && !diag) {
        const int64_t r = b0 + (tid - kT);
        if (r < a.n) a.adj[r * W + ti] = colbits[tid - kT];
    }
    if (tid == 0) {
        Prob &pw = bt.probs[d];
        if (wg_removed) add_ll(&pw.removed[0], (long long)wg_removed);
        if (wg_rechecks) add_ll(&pw.rechecks[0], (long long)wg_rechecks);
        if (ti == 0 && tj == 0) pw.tests[0] = (long long)(a.n * (a.n - 1) / 2);
    }
}

// Level 0 on a correlation matrix the caller supplied (FP64, no data): one work-group per row, a
// wavefront per 64-column word. Pair (i, j) is decided on C[min(i,j), max(i,j)], so both bits of a
// pair always agree; |atanh c| <= tau_0 removes it (Sec. 3.2, Eq. 5-6), as on the FP64 data path.
__global__ __launch_bounds__(256) void k_level0_given(Batch b) {
    const long long grow = blockIdx.x;
    const int d = find_base(b.row_base, b.count, grow);
    Prob &P = b.probs[d];
    const int64_t n = P.n, W = P.W, row = grow - b.row_base[d];
    const double *C = static_cast<const double *>(P.C);
    const double tau0 = P.tau[0];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int removed = 0;
    for (int64_t w = wave; w < W; w += 4) {
        const int64_t j = 64 * w + lane;
        bool keep = false;
        if (j < n && j != row) {
            const int64_t lo = row < j ? row : j, hi = row < j ? j : row;
            keep = !(fisher_z(C[lo * n + hi]) <= tau0);
            removed += (!keep && row < j) ? 1 : 0;
        }
        const unsigned long long bits = __ballot(keep);
        if (lane == 0) P.adj[row * W + w] = bits;
    }
    for (int o = 32; o >= 1; o >>= 1) removed += __shfl_xor(removed, o, 64);
    if (lane == 0 && removed) add_ll(&P.removed[0], (long long)removed);
    if (row == 0 && threadIdx.x == 0) P.tests[0] = (long long)(n * (n - 1) / 2);
}

hipError_t launch_level0_given(hipStream_t s, const Batch &b) {
    hipLaunchKernelGGL(k_level0_given, dim3((unsigned)b.total_rows), dim3(256), 0, s, b);
    return hipGetLastError();
}

// Deep staging (64 samples per barrier) when the tiles do not fill the CUs, or on BF16x3, whose
// three products per block keep a CU busy long enough to cover the loads of the next group.
hipError_t launch_corr(hipStream_t s, const Batch &b, long long tiles, int num_cu) {
    const dim3 grid((unsigned)tiles);
    const bool deep = tiles <= num_cu;
    if (b.prec == PC_PREC_FP64) {
        if (deep) hipLaunchKernelGGL((k_corr<PC_PREC_FP64, 4>), grid, dim3(256), 0, s, b);
        else hipLaunchKernelGGL((k_corr<PC_PREC_FP64, 1>), grid, dim3(256), 0, s, b);
    } else if (b.prec == PC_PREC_FP32) {
        if (deep) hipLaunchKernelGGL((k_corr<PC_PREC_FP32, 4>), grid, dim3(256), 0, s, b);
        else hipLaunchKernelGGL((k_corr<PC_PREC_FP32, 1>), grid, dim3(256), 0, s, b);
    } else {
        hipLaunchKernelGGL((k_corr<PC_PREC_BF16X3, 2>), grid, dim3(256), 0, s, b);
    }
    return hipGetLastError();
}

}  // namespace pcg
