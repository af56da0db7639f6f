// FP64 re-check of the CI tests whose FP32 decision fell inside the error band: Eq. 3-6 evaluated
// in FP64 from the standardized data, one queued test at a time.
#include "pc_level.h"

namespace pcg {

// ---------------------------------------------------------------------------------------------
// FP64 re-check
// ---------------------------------------------------------------------------------------------
constexpr int kRcThreads = 256;            // re-check work-group: 4 wavefronts per queued test

// After a queue overflow at level L the level loop stops and nothing clears the queue, which keeps
// level L's tests: the re-check launches of the levels after L (already enqueued) have none of
// their own, and must not read L's entries as tests of their level.
__device__ inline bool stale_queue(const Batch &b, int level) {
    const int ovf = __hip_atomic_load(&b.st->rq_overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return ovf != 0 && level > ovf;
}

// Queued tests of levels up to 14 (at most 16 variables). The FP64 Gram block of the standardized
// rows (i, j, S) is one 16 x 16 tile Z Z^T (gram_part); rows past l + 2 stay zero. On the FP64 path
// the block is read from C. With few queued tests a work-group takes each one and its four
// wavefronts split the samples (a quarter of the product chain each, partial tiles summed in LDS);
// with many, each wavefront takes its own test.
__global__ __launch_bounds__(kRcThreads) void k_recheck(Batch b, int level) {
    constexpr int kW = kRcThreads / 64;
    __shared__ double G[kW][16 * 16];
    __shared__ double part[kW][16 * 16];
    __shared__ double work[kW][kWorks];
    __shared__ int s_v[kW][16];
    __shared__ int s_prob, s_cls;
    if (stale_queue(b, level)) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const RqView view(b);
    const long long count = view.total();
    const int l = level, k = l + 2;
    RcStats rs;
    if (count <= 2 * (long long)gridDim.x) {
        double *Gw = G[0];
        int *vw = s_v[0];
        for (long long e = blockIdx.x; e < count; e += gridDim.x) {
            const RqEntry *qe = b.rq + view.index(e);
            if (tid < 16) vw[tid] = tid == 0 ? qe->i : (tid == 1 ? qe->j : (tid < k ? (int)qe->S[tid - 2] : -1));
            if (tid == 0) {
                s_prob = qe->prob;
                s_cls = qe->cls;
            }
            __syncthreads();
            const int prob = s_prob;
            Prob &P = b.probs[prob];
            if (b.prec != PC_PREC_FP64 && k <= 4) {
                double sp[6];
                gram_small_part(P, vw, k, lane, 128 * wave, 128 * kW, sp);
#pragma unroll
                for (int q = 0; q < 6; ++q) sp[q] = wave_sum64(sp[q]);
                if (lane == 0)
#pragma unroll
                    for (int q = 0; q < 6; ++q) part[wave][q] = sp[q];
                __syncthreads();
                if (tid == 0) {
                    double tot[6];
#pragma unroll
                    for (int q = 0; q < 6; ++q) tot[q] = (part[0][q] + part[1][q]) + (part[2][q] + part[3][q]);
                    gram_small_store(tot, k, Gw);
                }
            } else if (b.prec != PC_PREC_FP64) {
                const doublex4 acc = gram_part(P, vw[lane & 15], lane, 256 * wave, 256 * kW);
#pragma unroll
                for (int t = 0; t < 4; ++t) part[wave][((lane >> 4) + 4 * t) * 16 + (lane & 15)] = acc[t];
                __syncthreads();
                for (int q = tid; q < 256; q += kRcThreads) {
                    const int rr = q >> 4, cc = q & 15;
                    Gw[q] = rr == cc ? 1.0 : (part[0][q] + part[1][q]) + (part[2][q] + part[3][q]);
                }
            } else {
                for (int q = tid; q < k * k; q += kRcThreads) {
                    const int rr = q / k, cc = q % k;
                    Gw[rr * 16 + cc] = rr == cc ? 1.0 : static_cast<const double *>(P.C)[(int64_t)vw[rr] * P.n + vw[cc]];
                }
            }
            __syncthreads();
            if (wave == 0) {
                const int res = decide_wave<16>(Gw, 16, l, P.tau[l], work[0], kMMs, lane);
                if (lane == 0) {
                    rs.at(b, l, prob);
                    settle_recheck(b, P, l, res, vw[0], vw[1], s_cls, vw + 2, rs);
                }
            }
            __syncthreads();
        }
    } else {
        double *Gw = G[wave];
        int *vw = s_v[wave];
        for (long long e = (long long)blockIdx.x * kW + wave; e < count; e += (long long)gridDim.x * kW) {
            const RqEntry *qe = b.rq + view.index(e);
            if (lane < 16) vw[lane] = lane == 0 ? qe->i : (lane == 1 ? qe->j : (lane < k ? (int)qe->S[lane - 2] : -1));
            const int prob = qe->prob, cls = qe->cls;
            wave_sync();
            Prob &P = b.probs[prob];
            if (b.prec != PC_PREC_FP64 && k <= 4) {
                double sp[6];
                gram_small_part(P, vw, k, lane, 0, 128, sp);
#pragma unroll
                for (int q = 0; q < 6; ++q) sp[q] = wave_sum64(sp[q]);
                if (lane == 0) gram_small_store(sp, k, Gw);
            } else if (b.prec != PC_PREC_FP64) {
                const doublex4 acc = gram_part(P, vw[lane & 15], lane, 0, 256);
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
            const int res = decide_wave<16>(Gw, 16, l, P.tau[l], work[wave], kMMs, lane);
            if (lane == 0) {
                rs.at(b, l, prob);
                settle_recheck(b, P, l, res, vw[0], vw[1], cls, vw + 2, rs);
            }
            wave_sync();
        }
    }
    if (lane == 0) rs.flush(b, l);
}

// Queued tests of deeper levels (17 to 32 variables): one work-group per test. The Gram block
// spans 2 x 2 tiles of 16 x 16; wavefront w accumulates tile (w / 2, w % 2) over all samples, in
// rounds of 2 x 64 samples with one accumulator per round.
__global__ __launch_bounds__(kRcThreads) void k_recheck_deep(Batch b, int level) {
    __shared__ double part[kRcThreads / 64][16 * 16];
    __shared__ double G[kGramLd * kGramLd];
    __shared__ double work[kWork];
    __shared__ int s_v[32];        // variables of the tile rows: i, j, S..., then -1
    __shared__ int s_prob, s_cls;
    if (stale_queue(b, level)) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const RqView view(b);
    const long long count = view.total();
    const int l = level, k = l + 2;
    RcStats rs;
    for (long long e = blockIdx.x; e < count; e += gridDim.x) {
        const RqEntry *qe = b.rq + view.index(e);
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
            doublex4 acc[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) acc[q] = doublex4{0.0, 0.0, 0.0, 0.0};
            for (int64_t x0 = 0; x0 < mp; x0 += 2 * 64) {
                double va[2][kRcChunk], vb[2][kRcChunk];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int64_t x = x0 + 64 * q + off;
                    const bool in = x < mp;
#pragma unroll
                    for (int u = 0; u < kRcChunk; ++u) {
                        va[q][u] = ra >= 0 && in ? za[x + u] : 0.0;
                        vb[q][u] = rb >= 0 && in ? zb[x + u] : 0.0;
                    }
                }
#pragma unroll
                for (int u = 0; u < kRcChunk; ++u)
#pragma unroll
                    for (int q = 0; q < 2; ++q)
                        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(va[q][u], vb[q][u], acc[q], 0, 0, 0);
            }
            const doublex4 sum = acc[0] + acc[1];
#pragma unroll
            for (int t = 0; t < 4; ++t) part[wave][((lane >> 4) + 4 * t) * 16 + (lane & 15)] = sum[t];
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
        if (wave == 0) {
            const int res = decide_wave<32>(G, kGramLd, l, P.tau[l], work, kMM, lane);
            if (lane == 0) {
                rs.at(b, l, prob);
                settle_recheck(b, P, l, res, s_v[0], s_v[1], s_cls, s_v + 2, rs);
            }
        }
        __syncthreads();
    }
    if (tid == 0) rs.flush(b, l);
}

int recheck_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_recheck, kRcThreads, 0) != hipSuccess) return 0;
    return nb;
}

hipError_t launch_recheck(hipStream_t s, const Batch &b, int level, int grid) {
    if (level + 2 <= 16)
        hipLaunchKernelGGL(k_recheck, dim3(grid), dim3(kRcThreads), 0, s, b, level);
    else
        hipLaunchKernelGGL(k_recheck_deep, dim3(grid), dim3(kRcThreads), 0, s, b, level);
    return hipGetLastError();
}


}  // namespace pcg
