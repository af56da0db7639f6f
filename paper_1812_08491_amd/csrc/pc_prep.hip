// Data preparation: binomial table, run-state reset, column statistics and standardization.
//
// The paper takes the correlation matrix C as given (Sec. 4.3: the CI tests need only C, m and
// alpha). Here C is built from the data: every variable is centred with a two-pass FP64 mean and
// scaled to unit Euclidean norm, Z[:,a] = (X[:,a] - mu_a) / sqrt(sum_r (X[r,a] - mu_a)^2), so that
// C = Z^T Z is the Pearson correlation. Z is stored variable-major (n rows of mp samples, zero
// padded to a multiple of 64) in FP64 for re-checks, plus the low-precision copy the GEMM reads.
#include "pc_dev.h"

namespace pcg {

// Row a of Pascal's triangle by the multiplicative recurrence C(a,b+1) = C(a,b)(a-b)/(b+1),
// saturating at 2^62.
__global__ void k_binom(unsigned long long *binom, int64_t rows) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= rows) return;
    unsigned long long c = 1;
    for (int b = 0; b < kBinomCols; ++b) {
        binom[a * kBinomCols + b] = c;
        if (b >= a) {
            c = 0;
        } else if (c >= kSat) {
            c = kSat;
        } else {
            const unsigned long long f = (unsigned long long)(a - b);
            if (c > kSat / f) {
                c = kSat;
            } else {
                c = c * f / (unsigned long long)(b + 1);
                if (c > kSat) c = kSat;
            }
        }
    }
}

hipError_t launch_binom(hipStream_t s, unsigned long long *binom, int64_t rows) {
    hipLaunchKernelGGL(k_binom, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, binom, rows);
    return hipGetLastError();
}

// Zeroes the batch queue state and every problem's statistics and SepSet counter (one work-group
// per problem).
__global__ __launch_bounds__(256) void k_init(Batch b) {
    const int d = blockIdx.x, tid = threadIdx.x;
    if (d == 0 && tid < (int)(sizeof(DevState) / sizeof(int))) reinterpret_cast<int *>(b.st)[tid] = 0;
    Prob &p = b.probs[d];
    if (tid < kLevels) {
        p.tests[tid] = 0;
        p.removed[tid] = 0;
        p.rechecks[tid] = 0;
        p.items[tid] = 0;
        p.audit_viol[tid] = 0;
        p.probe_tests[tid] = 0;
        p.probe_removed[tid] = 0;
        p.maxdeg[tid] = 0;
    }
    if (tid == 0) {
        p.err = 0;
        p.tail_next = 0;
        p.tail_done = 0;
        if (p.rec_count) *p.rec_count = 0;
    }
}

hipError_t launch_init(hipStream_t s, const Batch &b) {
    hipLaunchKernelGGL(k_init, dim3((unsigned)b.count), dim3(256), 0, s, b);
    return hipGetLastError();
}

// Re-arms the level machinery before a caller-driven level: clears the stop flag and the queue
// counters (the problems' statistics are part of the freshly uploaded table).
__global__ void k_rearm(Batch b) {
    if (threadIdx.x < (int)(sizeof(DevState) / sizeof(int))) reinterpret_cast<int *>(b.st)[threadIdx.x] = 0;
}

hipError_t launch_rearm(hipStream_t s, const Batch &b) {
    hipLaunchKernelGGL(k_rearm, dim3(1), dim3(64), 0, s, b);
    return hipGetLastError();
}

// One work-group per 16 consecutive variables of one problem: 16 row groups x 16 columns, rows
// strided by 16, so each row group reads 128 contiguous bytes of X per step.
__global__ __launch_bounds__(256) void k_colstats(Batch b) {
    __shared__ double part[16][kCsCols];
    __shared__ int bad[kCsCols];
    const int d = find_base(b.cs_base, b.count, blockIdx.x);
    Prob &P = b.probs[d];
    const int64_t n = P.n, m = P.m;
    const double *__restrict__ X = P.X;
    const int c = threadIdx.x & (kCsCols - 1), g = threadIdx.x / kCsCols;
    const int64_t a = (int64_t)(blockIdx.x - b.cs_base[d]) * kCsCols + c;
    const bool valid = a < n;
    double s = 0.0;
    int nonfinite = 0;
    if (valid)
#pragma unroll 8
        for (int64_t r = g; r < m; r += 16) {
            const double x = X[r * n + a];
            nonfinite |= !isfinite(x);
            s += x;
        }
    part[g][c] = s;
    if (g == 0) bad[c] = 0;
    __syncthreads();
    if (nonfinite) atomicOr(&bad[c], 1);
    double tot = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) tot += part[k][c];
    const double mean = tot / (double)m;
    __syncthreads();
    double ss = 0.0;
    if (valid)
#pragma unroll 8
        for (int64_t r = g; r < m; r += 16) {
            const double dx = X[r * n + a] - mean;
            ss += dx * dx;
        }
    part[g][c] = ss;
    __syncthreads();
    if (g == 0 && valid) {
        double sst = 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) sst += part[k][c];
        P.mu[a] = mean;
        if (bad[c]) {
            P.inv[a] = 0.0;
            atomicCAS(&P.err, 0, (int)PC_ERR_NONFINITE);
        } else if (!(sst > 0.0)) {
            P.inv[a] = 0.0;
            atomicCAS(&P.err, 0, (int)PC_ERR_CONSTANT_COLUMN);
        } else {
            P.inv[a] = 1.0 / sqrt(sst);
        }
    }
}

hipError_t launch_colstats(hipStream_t s, const Batch &b, long long blocks) {
    hipLaunchKernelGGL(k_colstats, dim3((unsigned)blocks), dim3(256), 0, s, b);
    return hipGetLastError();
}

__device__ inline uint16_t bf16_bits_rne(float x) {
    uint32_t u = __float_as_uint(x);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;  // round to nearest even (inputs are finite)
    return (uint16_t)(u >> 16);
}

__device__ inline float bf16_bits_to_float(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Transposes a 64 x 64 tile of X (rows r, columns a) through LDS into Z (rows a, columns r).
// FP32 precision: zlo holds float; BF16x3: zhi/zlo hold the halves hi = bf16(z), lo = bf16(z - hi).
__global__ __launch_bounds__(256) void k_standardize(Batch b) {
    __shared__ double tile[64][65];
    const int d = find_base(b.st_base, b.count, blockIdx.x);
    Prob &P = b.probs[d];
    const int64_t n = P.n, m = P.m, mp = P.mp;
    const int64_t k = blockIdx.x - b.st_base[d], rblocks = mp / 64;
    const int64_t a0 = (k / rblocks) * 64, r0 = (k % rblocks) * 64;
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t a = a0 + c;
    // The tile's 16 loads per thread are issued together with the column's mean and scale.
    double xv[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int64_t r = r0 + g + 4 * t;
        xv[t] = a < n && r < m ? P.X[r * n + a] : 0.0;
    }
    double mua = 0.0, inva = 0.0;
    if (a < n) { mua = P.mu[a]; inva = P.inv[a]; }
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int64_t r = r0 + g + 4 * t;
        tile[g + 4 * t][c] = a < n && r < m ? (xv[t] - mua) * inva : 0.0;
    }
    __syncthreads();
    for (int aa = g; aa < 64; aa += 4) {
        const int64_t arow = a0 + aa;
        if (arow >= n) continue;
        const int64_t r = r0 + c;
        const double z = tile[c][aa];
        const size_t off = (size_t)arow * mp + r;
        P.zt64[off] = z;
        if (b.prec == PC_PREC_FP32) {
            static_cast<float *>(P.zlo)[off] = (float)z;
        } else if (b.prec == PC_PREC_BF16X3) {
            const uint16_t hi = bf16_bits_rne((float)z);
            const uint16_t lo = bf16_bits_rne((float)(z - (double)bf16_bits_to_float(hi)));
            static_cast<uint16_t *>(P.zhi)[off] = hi;
            static_cast<uint16_t *>(P.zlo)[off] = lo;
        }
    }
}

hipError_t launch_standardize(hipStream_t s, const Batch &b, long long blocks) {
    hipLaunchKernelGGL(k_standardize, dim3((unsigned)blocks), dim3(256), 0, s, b);
    return hipGetLastError();
}

}  // namespace pcg
