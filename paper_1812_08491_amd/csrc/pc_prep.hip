// Data preparation: run-state reset, binomial table, column statistics and standardization.
//
// The paper takes the correlation matrix C as given (Sec. 4.3: the CI tests need only C, m and
// alpha). Here C is built from the data: every variable is centred with a two-pass FP64 mean and
// scaled to unit Euclidean norm, Z[:,a] = (X[:,a] - mu_a) / sqrt(sum_r (X[r,a] - mu_a)^2), so that
// C = Z^T Z is the Pearson correlation. Z is stored variable-major (n rows of mp samples, zero
// padded to a multiple of 64) in FP64 for re-checks, plus the low-precision copy the GEMM reads.
#include <hip/hip_bf16.h>

#include "pc_dev.h"

namespace pcg {

__global__ void k_init(DevState *st, unsigned long long *binom, int64_t n, long long *zero_me) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a == 0) {
        // Zero the run state with vector stores.
        int *p = reinterpret_cast<int *>(st);
        for (size_t k = 0; k < sizeof(DevState) / sizeof(int); ++k) p[k] = 0;
        if (zero_me) *zero_me = 0;
    }
    if (a > n) return;
    // Row a of Pascal's triangle by the multiplicative recurrence C(a,b+1) = C(a,b)(a-b)/(b+1),
    // saturating at 2^62.
    unsigned long long c = 1;
    for (int b = 0; b < kBinomCols; ++b) {
        binom[a * kBinomCols + b] = c;
        if (b >= a) {
            c = 0;
        } else if (c >= kSat) {
            c = kSat;
        } else {
            unsigned long long f = (unsigned long long)(a - b);
            if (c > kSat / f) {
                c = kSat;
            } else {
                c = c * f / (unsigned long long)(b + 1);
                if (c > kSat) c = kSat;
            }
        }
    }
}

hipError_t launch_init(hipStream_t s, DevState *st, unsigned long long *binom, int64_t n,
                       long long *zero_me) {
    int64_t threads = n + 1;
    dim3 grid((unsigned)((threads + 255) / 256));
    hipLaunchKernelGGL(k_init, grid, dim3(256), 0, s, st, binom, n, zero_me);
    return hipGetLastError();
}

// Re-arms the level machinery before a caller-driven level: clears the stop flag and the
// per-level scratch counters (the statistics and the error flag are kept).
__global__ void k_rearm(DevState *st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->done = 0;
        st->blocks_done = 0u;
        st->deg_work = 0;
        st->rq_count = 0ull;
        st->rq_overflow = 0;
        st->overflow = 0;
    }
}

hipError_t launch_rearm(hipStream_t s, DevState *st) {
    hipLaunchKernelGGL(k_rearm, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

// One work-group per 64 consecutive variables: 4 row groups x 64 columns, rows strided by 4, so
// each row group reads 512 contiguous bytes of X per step.
__global__ __launch_bounds__(256) void k_colstats(const double *__restrict__ X, int64_t m, int64_t n,
                                                  double *__restrict__ mu, double *__restrict__ inv,
                                                  DevState *st) {
    __shared__ double part[4][64];
    __shared__ int bad[64];
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t a = (int64_t)blockIdx.x * 64 + c;
    const bool valid = a < n;
    double s = 0.0;
    int nonfinite = 0;
    if (valid)
        for (int64_t r = g; r < m; r += 4) {
            double x = X[r * n + a];
            nonfinite |= !isfinite(x);
            s += x;
        }
    part[g][c] = s;
    if (g == 0) bad[c] = 0;
    __syncthreads();
    if (nonfinite) atomicOr(&bad[c], 1);
    double mean = (part[0][c] + part[1][c] + part[2][c] + part[3][c]) / (double)m;
    __syncthreads();
    double ss = 0.0;
    if (valid)
        for (int64_t r = g; r < m; r += 4) {
            double d = X[r * n + a] - mean;
            ss += d * d;
        }
    part[g][c] = ss;
    __syncthreads();
    if (g == 0 && valid) {
        double tot = part[0][c] + part[1][c] + part[2][c] + part[3][c];
        mu[a] = mean;
        if (bad[c]) {
            inv[a] = 0.0;
            atomicCAS(&st->err, 0, (int)PC_ERR_NONFINITE);
        } else if (!(tot > 0.0)) {
            inv[a] = 0.0;
            atomicCAS(&st->err, 0, (int)PC_ERR_CONSTANT_COLUMN);
        } else {
            inv[a] = 1.0 / sqrt(tot);
        }
    }
}

hipError_t launch_colstats(hipStream_t s, const double *X, int64_t m, int64_t n, double *mu,
                           double *inv, DevState *st) {
    dim3 grid((unsigned)((n + 63) / 64));
    hipLaunchKernelGGL(k_colstats, grid, dim3(256), 0, s, X, m, n, mu, inv, st);
    return hipGetLastError();
}

__device__ inline uint16_t bf16_bits_rne(float x) {
    uint32_t u = __float_as_uint(x);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;  // round to nearest even (inputs are finite)
    return (uint16_t)(u >> 16);
}

__device__ inline float bf16_bits_to_float(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Transposes a 64 x 64 tile of X (rows r, columns a) through LDS into Z (rows a, columns r).
// prec selects the low-precision copy: FP32 -> zlo as float; BF16x3 -> zhi/zlo as the two BF16
// halves hi = bf16(z), lo = bf16(z - hi).
__global__ __launch_bounds__(256) void k_standardize(const double *__restrict__ X, int64_t m,
                                                     int64_t n, int64_t mp,
                                                     const double *__restrict__ mu,
                                                     const double *__restrict__ inv,
                                                     double *__restrict__ zt64, void *zlo,
                                                     void *zhi, int prec) {
    __shared__ double tile[64][65];
    const int64_t a0 = (int64_t)blockIdx.x * 64, r0 = (int64_t)blockIdx.y * 64;
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t a = a0 + c;
    double mua = 0.0, inva = 0.0;
    if (a < n) { mua = mu[a]; inva = inv[a]; }
    for (int rr = g; rr < 64; rr += 4) {
        int64_t r = r0 + rr;
        double z = 0.0;
        if (a < n && r < m) z = (X[r * n + a] - mua) * inva;
        tile[rr][c] = z;
    }
    __syncthreads();
    for (int aa = g; aa < 64; aa += 4) {
        int64_t arow = a0 + aa;
        if (arow >= n) continue;
        int64_t r = r0 + c;
        double z = tile[c][aa];
        size_t off = (size_t)arow * mp + r;
        zt64[off] = z;
        if (prec == PC_PREC_FP32) {
            static_cast<float *>(zlo)[off] = (float)z;
        } else if (prec == PC_PREC_BF16X3) {
            float zf = (float)z;
            uint16_t hi = bf16_bits_rne(zf);
            float rem = (float)(z - (double)bf16_bits_to_float(hi));
            uint16_t lo = bf16_bits_rne(rem);
            static_cast<uint16_t *>(zhi)[off] = hi;
            static_cast<uint16_t *>(zlo)[off] = lo;
        }
    }
}

hipError_t launch_standardize(hipStream_t s, const double *X, int64_t m, int64_t n, int64_t mp,
                              const double *mu, const double *inv, double *zt64, void *zlo,
                              void *zhi, int prec) {
    dim3 grid((unsigned)((n + 63) / 64), (unsigned)(mp / 64));
    hipLaunchKernelGGL(k_standardize, grid, dim3(256), 0, s, X, m, n, mp, mu, inv, zt64, zlo, zhi,
                       prec);
    return hipGetLastError();
}

}  // namespace pcg
