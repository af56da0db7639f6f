// Learned conditioning-set ordering: candidate features, a small MLP (forward, backward, Adam) and
// the probe pass that tests each edge's best-scored subsets first.
//
// PC-stable's result does not depend on the order in which conditioning sets are tried (Sec. 2.4:
// S is drawn from the snapshot G', removals go to G). So a level can first test, for every edge,
// the few subsets built from the candidates a model ranks highest, and then run the plain
// enumeration on the same G': edges the probe removed are skipped by the live-bit check of the
// plain kernel, and the adjacency after the level is the same as without the probe.
//
// Features of candidate k for the directed edge (i, j), all from quantities the method computes:
//   |C_ij|, |C_ik|, |C_jk|, |rho_ij.k| (the level-1 partial correlation), d_i/64, d_j/64, d_k/64,
//   l/8 (degrees in G' of the level).
// MLP: 8 -> 64 -> 64 -> 1 with ReLU; the 64 x 64 products run on v_mfma_f32_16x16x4f32.
#include "pc_citest.h"
#include "pc_comb.h"
#include "pc_dev.h"

namespace pcg {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kIn = PC_MLP_IN, kHid = PC_MLP_HID;
constexpr int oW1 = 0, oB1 = kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kHid;
static_assert(oB3 + 1 == PC_MLP_PARAMS, "parameter layout");
constexpr int kTile = 64;   // rows per work-group

struct MlpSmem {
    float W2[kHid][kHid + 1];
    float A[kTile][kHid + 1];   // H1 (forward) / H1 (backward)
    float B[kTile][kHid + 1];   // H2 (forward) / H2 then dZ1 (backward)
    float W1[kHid][kIn];
    float b1[kHid], b2[kHid], W3[kHid];
    float X[kTile][kIn];
    float b3;
};

__device__ inline void load_params(MlpSmem &sm, const float *p, int tid) {
    for (int e = tid; e < kHid * kHid; e += 256) sm.W2[e / kHid][e % kHid] = p[oW2 + e];
    for (int e = tid; e < kHid * kIn; e += 256) sm.W1[e / kIn][e % kIn] = p[oW1 + e];
    if (tid < kHid) {
        sm.b1[tid] = p[oB1 + tid];
        sm.b2[tid] = p[oB2 + tid];
        sm.W3[tid] = p[oW3 + tid];
    }
    if (tid == 0) sm.b3 = p[oB3];
}

// Forward of rows [r0, r0 + 64): H1 into sm.A, H2 into sm.B, scores out.
__device__ inline void mlp_tile_forward(MlpSmem &sm, const float *X, long long rows, long long r0,
                                        float *scores, float *act, int tid) {
    const int lane = tid & 63, wave = tid >> 6;
    const int r = tid >> 2, part = tid & 3;
    float x[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) x[k] = r0 + r < rows ? X[(r0 + r) * kIn + k] : 0.0f;
    if (part == 0) {
#pragma unroll
        for (int k = 0; k < kIn; ++k) sm.X[r][k] = x[k];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int o = part * 16 + u;
        float z = sm.b1[o];
#pragma unroll
        for (int k = 0; k < kIn; ++k) z += sm.W1[o][k] * x[k];
        sm.A[r][o] = z > 0.0f ? z : 0.0f;
    }
    __syncthreads();
    // H2 = relu(H1 W2^T + b2): wave w computes rows 16w..16w+15, all four 16-column blocks.
    floatx4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k4 = 0; k4 < kHid / 4; ++k4) {
        const float a = sm.A[16 * wave + (lane & 15)][4 * k4 + (lane >> 4)];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float bv = sm.W2[16 * c + (lane & 15)][4 * k4 + (lane >> 4)];
            acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc[c], 0, 0, 0);
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * wave + 4 * (lane >> 4) + v, col = 16 * c + (lane & 15);
            const float z = acc[c][v] + sm.b2[col];
            sm.B[row][col] = z > 0.0f ? z : 0.0f;
        }
    __syncthreads();
    float s = 0.0f;
#pragma unroll
    for (int u = 0; u < 16; ++u) s += sm.W3[part * 16 + u] * sm.B[r][part * 16 + u];
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    if (part == 0 && r0 + r < rows) scores[r0 + r] = s + sm.b3;
    if (act && r0 + r < rows) {
        for (int u = 0; u < 16; ++u) {
            act[(r0 + r) * 2 * kHid + part * 16 + u] = sm.A[r][part * 16 + u];
            act[(r0 + r) * 2 * kHid + kHid + part * 16 + u] = sm.B[r][part * 16 + u];
        }
    }
    __syncthreads();
}

// Row count from a device counter (feature rows of a level) or a fixed value.
__global__ __launch_bounds__(256) void k_mlp_fwd(const float *params, const float *X, long long rows,
                                                 const long long *rows_dev, long long rows_cap,
                                                 float *scores, float *act, const int *skip) {
    __shared__ MlpSmem sm;
    if (skip && *skip) return;
    long long nrows = rows_dev ? *rows_dev : rows;
    if (nrows > rows_cap) return;
    const int tid = threadIdx.x;
    load_params(sm, params, tid);
    __syncthreads();
    for (long long r0 = (long long)blockIdx.x * kTile; r0 < nrows; r0 += (long long)gridDim.x * kTile)
        mlp_tile_forward(sm, X, nrows, r0, scores, act, tid);
}

// Backward of rows [64 b, 64 b + 64) into a per-work-group partial gradient (deterministic sum
// afterwards). dscore = dLoss/dscore per row.
__global__ __launch_bounds__(256) void k_mlp_bwd(const float *params, const float *X, long long rows,
                                                 const float *act, const float *dscore, float *partial) {
    __shared__ MlpSmem sm;
    __shared__ float dZ2[kTile][kHid + 1];
    __shared__ float dS[kTile];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long r0 = (long long)blockIdx.x * kTile;
    float *g = partial + (long long)blockIdx.x * PC_MLP_PARAMS;
    load_params(sm, params, tid);
    {
        const int r = tid >> 2, part = tid & 3;
        const bool in = r0 + r < rows;
        for (int u = 0; u < 16; ++u) {
            const int o = part * 16 + u;
            sm.A[r][o] = in ? act[(r0 + r) * 2 * kHid + o] : 0.0f;
            sm.B[r][o] = in ? act[(r0 + r) * 2 * kHid + kHid + o] : 0.0f;
        }
        if (part == 0) {
            for (int k = 0; k < kIn; ++k) sm.X[r][k] = in ? X[(r0 + r) * kIn + k] : 0.0f;
            dS[r] = in ? dscore[r0 + r] : 0.0f;
        }
    }
    __syncthreads();
    {
        const int r = tid >> 2, part = tid & 3;
        for (int u = 0; u < 16; ++u) {
            const int o = part * 16 + u;
            dZ2[r][o] = sm.B[r][o] > 0.0f ? dS[r] * sm.W3[o] : 0.0f;
        }
    }
    __syncthreads();
    // dW3, db3, db2 (row sums).
    if (tid < kHid) {
        float s = 0.0f;
        for (int r = 0; r < kTile; ++r) s += dS[r] * sm.B[r][tid];
        g[oW3 + tid] = s;
    } else if (tid == kHid) {
        float s = 0.0f;
        for (int r = 0; r < kTile; ++r) s += dS[r];
        g[oB3] = s;
    } else if (tid >= 128 && tid < 128 + kHid) {
        const int o = tid - 128;
        float s = 0.0f;
        for (int r = 0; r < kTile; ++r) s += dZ2[r][o];
        g[oB2 + o] = s;
    }
    // dW2[o][i] = sum_r dZ2[r][o] H1[r][i] (wave w: o block w) and dH1[r][i] = sum_o dZ2[r][o] W2[o][i]
    // (wave w: row block w); K = 64 in both, on MFMA.
    floatx4 gw[4], gh[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) { gw[c] = floatx4{0.f, 0.f, 0.f, 0.f}; gh[c] = gw[c]; }
#pragma unroll
    for (int k4 = 0; k4 < kTile / 4; ++k4) {
        const float aw = dZ2[4 * k4 + (lane >> 4)][16 * wave + (lane & 15)];
        const float ah = dZ2[16 * wave + (lane & 15)][4 * k4 + (lane >> 4)];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float bw = sm.A[4 * k4 + (lane >> 4)][16 * c + (lane & 15)];
            const float bh = sm.W2[4 * k4 + (lane >> 4)][16 * c + (lane & 15)];
            gw[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(aw, bw, gw[c], 0, 0, 0);
            gh[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ah, bh, gh[c], 0, 0, 0);
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int o = 16 * wave + 4 * (lane >> 4) + v, i = 16 * c + (lane & 15);
            g[oW2 + o * kHid + i] = gw[c][v];
        }
    __syncthreads();  // every read of sm.B (H2) is done: it now holds dZ1
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 16 * wave + 4 * (lane >> 4) + v, i = 16 * c + (lane & 15);
            sm.B[r][i] = sm.A[r][i] > 0.0f ? gh[c][v] : 0.0f;
        }
    __syncthreads();
    if (tid < kHid) {
        float s = 0.0f;
        for (int r = 0; r < kTile; ++r) s += sm.B[r][tid];
        g[oB1 + tid] = s;
    }
    for (int e = tid; e < kHid * kIn; e += 256) {
        const int i = e / kIn, k = e % kIn;
        float s = 0.0f;
        for (int r = 0; r < kTile; ++r) s += sm.B[r][i] * sm.X[r][k];
        g[oW1 + e] = s;
    }
}

__global__ __launch_bounds__(256) void k_sum_partials(const float *partial, int nparts, float *grads) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= PC_MLP_PARAMS) return;
    float s = 0.0f;
    for (int w = 0; w < nparts; ++w) s += partial[(long long)w * PC_MLP_PARAMS + p];
    grads[p] = s;
}

// Weighted binary cross-entropy on logits, mean over rows: loss and dLoss/dscore.
__global__ __launch_bounds__(1024) void k_bce(const float *scores, const float *labels, long long rows,
                                              float pos_weight, float *dscore, double *loss) {
    __shared__ double part[1024];
    const int tid = threadIdx.x;
    double s = 0.0;
    const float inv = 1.0f / (float)rows;
    for (long long r = tid; r < rows; r += 1024) {
        const float z = scores[r], y = labels[r];
        const float sp_pos = fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z)));   // softplus(z)
        const float sp_neg = sp_pos - z;                                  // softplus(-z)
        s += (double)(pos_weight * y * sp_neg + (1.0f - y) * sp_pos);
        const float sig = 1.0f / (1.0f + expf(-z));
        dscore[r] = (pos_weight * y * (sig - 1.0f) + (1.0f - y) * sig) * inv;
    }
    part[tid] = s;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (tid < o) part[tid] += part[tid + o];
        __syncthreads();
    }
    if (tid == 0) *loss = part[0] / (double)rows;
}

__global__ __launch_bounds__(256) void k_adam(float *params, const float *grads, float *m1, float *m2,
                                              int step, float lr, float beta1, float beta2, float eps) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= PC_MLP_PARAMS) return;
    const float g = grads[p];
    const float a = beta1 * m1[p] + (1.0f - beta1) * g;
    const float b = beta2 * m2[p] + (1.0f - beta2) * g * g;
    m1[p] = a;
    m2[p] = b;
    const float ah = a / (1.0f - powf(beta1, (float)step));
    const float bh = b / (1.0f - powf(beta2, (float)step));
    params[p] -= lr * ah / (sqrtf(bh) + eps);
}

hipError_t launch_mlp_forward(hipStream_t s, const float *params, const float *X, long long rows,
                              const long long *rows_dev, long long rows_cap, float *scores, float *act,
                              const int *skip, int grid) {
    hipLaunchKernelGGL(k_mlp_fwd, dim3(grid), dim3(256), 0, s, params, X, rows, rows_dev, rows_cap, scores,
                       act, skip);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(hipStream_t s, const float *params, const float *X, long long rows,
                               const float *act, const float *dscore, float *partial, float *grads) {
    const int tiles = (int)((rows + kTile - 1) / kTile);
    hipLaunchKernelGGL(k_mlp_bwd, dim3(tiles), dim3(256), 0, s, params, X, rows, act, dscore, partial);
    hipLaunchKernelGGL(k_sum_partials, dim3((PC_MLP_PARAMS + 255) / 256), dim3(256), 0, s, partial, tiles, grads);
    return hipGetLastError();
}

hipError_t launch_bce(hipStream_t s, const float *scores, const float *labels, long long rows, float pos_weight,
                      float *dscore, double *loss) {
    hipLaunchKernelGGL(k_bce, dim3(1), dim3(1024), 0, s, scores, labels, rows, pos_weight, dscore, loss);
    return hipGetLastError();
}

hipError_t launch_adam(hipStream_t s, float *params, const float *grads, float *m1, float *m2, int step, float lr,
                       float beta1, float beta2, float eps) {
    hipLaunchKernelGGL(k_adam, dim3((PC_MLP_PARAMS + 255) / 256), dim3(256), 0, s, params, grads, m1, m2, step, lr,
                       beta1, beta2, eps);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Features
// ---------------------------------------------------------------------------------------------

// Exclusive offsets of the feature rows of each flattened row (d_i (d_i - 1) candidate pairs of
// the level's G'); foff[total_rows] is the total. Sets *skip when the total exceeds the capacity
// (the level then runs without a probe) or when the level has no work.
// per_node = 0: d(d - 1) rows per node (edge features); 1: d rows (candidate features of a node).
__global__ __launch_bounds__(1024) void k_feat_plan(Batch b, long long *foff, long long cap, int *skip, int per_node) {
    __shared__ long long part[1024 / 64];
    const int tid = threadIdx.x;
    if (b.st->done) {
        if (tid == 0) *skip = 1;
        return;
    }
    const long long N = b.total_rows;
    const long long chunk = (N + 1023) / 1024;
    const long long lo = tid * chunk, hi = lo + chunk < N ? lo + chunk : N;
    auto cnt = [&](long long k) -> long long {
        const int d = find_base(b.row_base, b.count, k);
        const long long dg = b.probs[d].deg[k - b.row_base[d]];
        return per_node ? dg : dg * (dg - 1);
    };
    long long s = 0;
    for (long long k = lo; k < hi; ++k) s += cnt(k);
    long long total = 0;
    long long run = block_exclusive_scan<1024>(s, part, total);
    for (long long k = lo; k < hi; ++k) {
        foff[k] = run;
        run += cnt(k);
    }
    if (tid == 0) {
        foff[N] = total;
        *skip = total > cap || total == 0 ? 1 : 0;
    }
}

// One work-group per flattened row i: the features of every (j = N_i[p], k = N_i[q], q != p).
// meta (optional) receives (i, j, k) per feature row.
template <typename T>
__global__ __launch_bounds__(256) void k_features(Batch b, int level, const long long *foff,
                                                  float *feats, int *meta, const int *skip) {
    if (*skip) return;
    const long long grow = blockIdx.x;
    const int pd = find_base(b.row_base, b.count, grow);
    const Prob &P = b.probs[pd];
    const int64_t n = P.n;
    const int row = (int)(grow - b.row_base[pd]);
    const int d = P.deg[row];
    if (d < 2) return;
    const T *C = static_cast<const T *>(P.C);
    const int *nb = P.nbr + (int64_t)row * n;
    const long long base = foff[grow];
    const long long cnt = (long long)d * (d - 1);
    const float di = (float)d / 64.0f, lv = (float)level / 8.0f;
    for (long long e = threadIdx.x; e < cnt; e += 256) {
        const int p = (int)(e / (d - 1)), qq = (int)(e % (d - 1));
        const int q = qq < p ? qq : qq + 1;
        const int j = nb[p], k = nb[q];
        const float cij = (float)C[(int64_t)row * n + j], cik = (float)C[(int64_t)row * n + k];
        const float cjk = (float)C[(int64_t)j * n + k];
        const float den = (1.0f - cik * cik) * (1.0f - cjk * cjk);
        const float rho = den > 0.0f ? (cij - cik * cjk) * rsqrtf(den) : 0.0f;
        float *f = feats + (base + e) * kIn;
        f[0] = fabsf(cij);
        f[1] = fabsf(cik);
        f[2] = fabsf(cjk);
        f[3] = fminf(fabsf(rho), 1.0f);
        f[4] = di;
        f[5] = (float)P.deg[j] / 64.0f;
        f[6] = (float)P.deg[k] / 64.0f;
        f[7] = lv;
        if (meta) {
            meta[(base + e) * 3 + 0] = row;
            meta[(base + e) * 3 + 1] = j;
            meta[(base + e) * 3 + 2] = k;
        }
    }
}

hipError_t launch_feat_plan(hipStream_t s, const Batch &b, long long *foff, long long cap, int *skip) {
    hipLaunchKernelGGL(k_feat_plan, dim3(1), dim3(1024), 0, s, b, foff, cap, skip, 0);
    return hipGetLastError();
}

hipError_t launch_features(hipStream_t s, const Batch &b, int level, const long long *foff, float *feats,
                           int *meta, const int *skip) {
    if (b.prec == PC_PREC_FP64)
        hipLaunchKernelGGL(k_features<double>, dim3((unsigned)b.total_rows), dim3(256), 0, s, b, level, foff,
                           feats, meta, skip);
    else
        hipLaunchKernelGGL(k_features<float>, dim3((unsigned)b.total_rows), dim3(256), 0, s, b, level, foff,
                           feats, meta, skip);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Probe: per directed edge, the subsets of its top-Q candidates, scored by the MLP in one kernel
// ---------------------------------------------------------------------------------------------
constexpr int kTopMax = 8;
constexpr int kProbeRowCap = 24;   // rows with more neighbours skip the probe (row block in LDS)
constexpr int kProbeThreads = 256;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// C(a, b) for a, b <= kTopMax (subsets of the top candidates).
struct TopBinom {
    __device__ unsigned long long operator()(int a, int b) const {
        if (b < 0 || a < b) return 0ull;
        unsigned long long c = 1;
#pragma unroll
        for (int k = 0; k < kTopMax; ++k)
            if (k < b) c = c * (unsigned long long)(a - k);
        unsigned long long f = 1;
#pragma unroll
        for (int k = 2; k <= kTopMax; ++k)
            if (k <= b) f *= (unsigned long long)k;
        return c / f;
    }
};

// Orders the LDS accesses of the lanes of one wavefront around a cooperative step.
__device__ inline void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Round-to-nearest-even BF16 bits of a finite float.
__device__ inline uint16_t bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

constexpr int kProbeStage = 256;   // independent probe tests of a row settled together

template <typename T>
struct __align__(16) ProbeSmem {
    uint16_t W1[kHid][8];              // layer-1 weights as the B operand rows ([out][in]), BF16
    uint16_t W2[kHid][kHid + 8];       // layer-2 weights ([out][in]), BF16, rows padded to 144 B
    uint16_t X[4][64][8];              // per wavefront: features of its 64 candidate rows
    uint16_t H1[4][16][kHid + 8];      // per wavefront: layer-1 activations of one 16-row tile
    float b1[kHid], b2[kHid], W3[kHid];
    float b3;
    float sc[kProbeRowCap * (kProbeRowCap - 1)];   // MLP score of every (p, q != p) of the row
    T blk[kProbeRowCap][kProbeRowCap + 1];         // C[N_i, N_i]
    T ci[kProbeRowCap];                            // C[i, N_i]
    int nb[kProbeRowCap];
    float dg[kProbeRowCap];
    int live[kProbeRowCap];                        // edge (i, N_i[p]) still in G at the test phase
    unsigned char top[kProbeRowCap][kTopMax];      // best candidate positions of each edge, by rank
    int stage[kProbeStage];                        // (p, subset) of the independent tests
    int nstage, nwin;
    unsigned long long rec_base;
    long long tests, removed;
};

// One work-group per row i of G' (grid-stride, persistent), for rows with L + 1 <= d_i <= 48
// (the row's block C[N_i, N_i], C[i, N_i] and all scores are staged in LDS):
//  1. the MLP scores every candidate k = N_i[q] of every directed edge (i, N_i[p]), q != p: each
//     wavefront takes 64 candidate rows at a time, computes their features in FP32, and runs the
//     8 -> 64 -> 64 -> 1 network on v_mfma_f32_16x16x32_bf16 in 16-row tiles (layer 1 with K
//     padded to 32, layer 2 in two K-steps; BF16 weights and activations, FP32 accumulation), the
//     last layer as a reduction over the 16 lanes that hold a candidate's hidden units;
//  2. every candidate row counts the candidates of its edge that score higher (ties: lower
//     position first); those with rank < Q = min(top, d_i - 1) are the edge's top candidates;
//  3. the threads share the (live edge, subset of its top-Q) pairs and test them with the FP32
//     test of the level kernel (same band, same re-check queue); the independent ones are staged
//     and settled together: the atomic AND on the edge bit picks one winner per edge, and the
//     winners take consecutive SepSet slots with one atomic add.
template <typename T, int L>
__global__ __launch_bounds__(kProbeThreads) void k_probe(Batch b, const float *params, int topq) {
    __shared__ ProbeSmem<T> sm;
    if (b.st->done) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // Parameters: BF16 weights, FP32 biases.
    for (int e = tid; e < kHid * kIn; e += kProbeThreads) sm.W1[e / kIn][e % kIn] = bf16_rne(params[oW1 + e]);
    for (int e = tid; e < kHid * kHid; e += kProbeThreads) sm.W2[e / kHid][e % kHid] = bf16_rne(params[oW2 + e]);
    if (tid < kHid) {
        sm.b1[tid] = params[oB1 + tid];
        sm.b2[tid] = params[oB2 + tid];
        sm.W3[tid] = params[oW3 + tid];
    }
    if (tid == 0) {
        sm.b3 = params[oB3];
        sm.tests = 0;
        sm.removed = 0;
        sm.nstage = 0;
        sm.nwin = 0;
    }
    int stats_pd = -1;
    for (long long grow = blockIdx.x; grow < b.total_rows; grow += gridDim.x) {
        const int pd = find_base(b.row_base, b.count, grow);
        Prob &P = b.probs[pd];
        const int row = (int)(grow - b.row_base[pd]);
        const int d = P.deg[row];
        if (d < L + 1 || d > kProbeRowCap || !(L <= P.max_level && P.tau[L] == P.tau[L])) continue;
        __syncthreads();   // the previous row's LDS contents and statistics are no longer read
        if (tid == 0 && pd != stats_pd) {
            if (stats_pd >= 0) {
                Prob &Ps = b.probs[stats_pd];
                if (sm.tests) { add_ll(&Ps.tests[L], sm.tests); add_ll(&Ps.probe_tests[L], sm.tests); }
                if (sm.removed) { add_ll(&Ps.removed[L], sm.removed); add_ll(&Ps.probe_removed[L], sm.removed); }
            }
            sm.tests = 0;
            sm.removed = 0;
        }
        stats_pd = pd;
        const int64_t n = P.n, W = P.W;
        const T *C = static_cast<const T *>(P.C);
        const int *nbg = P.nbr + (int64_t)row * n;
        if (tid < d) {
            const int k = nbg[tid];
            sm.nb[tid] = k;
            sm.dg[tid] = (float)P.deg[k] / 64.0f;
            sm.ci[tid] = C[(int64_t)row * n + k];
        }
        __syncthreads();
        // The row's block C[N_i, N_i], every gather issued before any store.
        {
            constexpr int kPer = (kProbeRowCap * kProbeRowCap + kProbeThreads - 1) / kProbeThreads;
            T v[kPer];
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int e = tid + u * kProbeThreads;
                v[u] = (T)0;
                if (e < d * d) v[u] = C[(int64_t)sm.nb[e / d] * n + sm.nb[e % d]];
            }
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int e = tid + u * kProbeThreads;
                if (e < d * d) sm.blk[e / d][e % d] = v[u];
            }
        }
        __syncthreads();
        const float di = (float)d / 64.0f, lv = (float)L / 8.0f;
        const int ncand = d - 1, nrows = d * ncand;
        // 1. Scores: 64 candidate rows per wavefront pass.
        for (int b0 = 64 * wave; b0 < nrows; b0 += 256) {
            {
                const int r = b0 + lane;
                float x[kIn] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                if (r < nrows) {
                    const int p = r / ncand, qq = r - p * ncand, q = qq < p ? qq : qq + 1;
                    const float cij = (float)sm.ci[p], cik = (float)sm.ci[q], cjk = (float)sm.blk[p][q];
                    const float den = (1.0f - cik * cik) * (1.0f - cjk * cjk);
                    const float rho = den > 0.0f ? (cij - cik * cjk) * rsqrtf(den) : 0.0f;
                    x[0] = fabsf(cij);
                    x[1] = fabsf(cik);
                    x[2] = fabsf(cjk);
                    x[3] = fminf(fabsf(rho), 1.0f);
                    x[4] = di;
                    x[5] = sm.dg[p];
                    x[6] = sm.dg[q];
                    x[7] = lv;
                }
#pragma unroll
                for (int u = 0; u < kIn; ++u) sm.X[wave][lane][u] = bf16_rne(x[u]);
            }
            wave_sync_lds();
            const bf16x8 zero8 = {};
            const int tiles = (nrows - b0 + 15) / 16 < 4 ? (nrows - b0 + 15) / 16 : 4;
            for (int mt = 0; mt < tiles; ++mt) {
                // Layer 1: H1 = relu(X W1^T + b1); only lanes 0-15 carry K (the 8 features).
                const bf16x8 ax = lane < 16 ? *reinterpret_cast<const bf16x8 *>(&sm.X[wave][16 * mt + lane][0]) : zero8;
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const bf16x8 bw = lane < 16 ? *reinterpret_cast<const bf16x8 *>(&sm.W1[16 * nt + lane][0]) : zero8;
                    const floatx4 z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, bw, floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                    const int col = 16 * nt + (lane & 15);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const float h = z[v] + sm.b1[col];
                        sm.H1[wave][4 * (lane >> 4) + v][col] = bf16_rne(h > 0.0f ? h : 0.0f);
                    }
                }
                wave_sync_lds();
                // Layer 2: H2 = relu(H1 W2^T + b2), K = 64 in two steps of 32.
                floatx4 acc[4];
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) acc[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    const bf16x8 ah = *reinterpret_cast<const bf16x8 *>(&sm.H1[wave][lane & 15][32 * ks + 8 * (lane >> 4)]);
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) {
                        const bf16x8 bw =
                            *reinterpret_cast<const bf16x8 *>(&sm.W2[16 * nt + (lane & 15)][32 * ks + 8 * (lane >> 4)]);
                        acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bw, acc[nt], 0, 0, 0);
                    }
                }
                wave_sync_lds();   // H1 of this tile is read; the next tile may overwrite it
                // Layer 3: score = W3 . H2 + b3; lane l holds rows 4 (l / 16) + v, column l % 16 of
                // each 16-column block, so the 16 lanes of a row group reduce together.
                float part[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    float sacc = 0.0f;
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) {
                        const int col = 16 * nt + (lane & 15);
                        const float h = acc[nt][v] + sm.b2[col];
                        sacc += (h > 0.0f ? h : 0.0f) * sm.W3[col];
                    }
                    part[v] = sacc;
                }
#pragma unroll
                for (int o = 1; o < 16; o <<= 1)
#pragma unroll
                    for (int v = 0; v < 4; ++v) part[v] += __shfl_xor(part[v], o, 64);
                if ((lane & 15) == 0)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = b0 + 16 * mt + 4 * (lane >> 4) + v;
                        if (r < nrows) sm.sc[r] = part[v] + sm.b3;
                    }
            }
        }
        // Live bits of the row's edges, read once the scores are done (removals made meanwhile by
        // other work-groups are seen).
        if (tid < d) {
            const int j = sm.nb[tid];
            sm.live[tid] = (int)((live_word(P.adj + (int64_t)row * W + (j >> 6)) >> (j & 63)) & 1ull);
        }
        __syncthreads();
        // 2. Rank of every candidate row within its edge; the top Q are kept.
        const int Q = topq < ncand ? topq : ncand;
        for (int r = tid; r < nrows; r += kProbeThreads) {
            const int p = r / ncand, qq = r - p * ncand;
            const float s0 = sm.sc[r];
            const float *seg = sm.sc + p * ncand;
            int rank = 0;
            for (int u = 0; u < ncand; ++u) {
                const float su = seg[u];
                rank += (su > s0 || (su == s0 && u < qq)) ? 1 : 0;
            }
            if (rank < Q) sm.top[p][rank] = (unsigned char)(qq < p ? qq : qq + 1);
        }
        __syncthreads();
        // 3. The C(Q, L) subsets of the top candidates of every live edge.
        const double tau = P.tau[L];
        const float tl = P.t[L], band = P.band[L];
        const int nsub = (int)TopBinom()(Q, L);
        auto CS = [&](int a, int c) -> T { return a == c ? (T)1 : sm.blk[a][c]; };
        auto CI = [&](int a) -> T { return sm.ci[a]; };
        // Positions of subset s of edge p, in ascending order (so S is in id order).
        auto subset = [&](int p, int s, int (&P_)[L]) {
            int idx[L];
            comb_unrank<L>(Q, (unsigned long long)s, idx, TopBinom());
#pragma unroll
            for (int c = 0; c < L; ++c) P_[c] = sm.top[p][idx[c]];
#pragma unroll
            for (int u = 1; u < L; ++u)
#pragma unroll
                for (int v = u; v > 0; --v)
                    if (P_[v - 1] > P_[v]) { const int t = P_[v]; P_[v] = P_[v - 1]; P_[v - 1] = t; }
        };
        long long my_tests = 0;
        for (int e = tid; e < d * nsub; e += kProbeThreads) {
            const int p = e / nsub, si = e - p * nsub;
            if (!sm.live[p]) continue;
            int P_[L];
            subset(p, si, P_);
            SetFactor<T, L> f;
            f.build(P_, CS, CI);
            ++my_tests;
            const int dec = f.test(P_, p, CS, CI, tau, tl, band);
            if (dec == 2) {
                int sid[L];
#pragma unroll
                for (int c = 0; c < L; ++c) sid[c] = sm.nb[P_[c]];
                push_recheck<L>(b, pd, row, sm.nb[p], sid, 2);
            } else if (dec == 1) {
                const int slot = atomicAdd(&sm.nstage, 1);
                if (slot < kProbeStage) {
                    sm.stage[slot] = e;
                } else {
                    const int j = sm.nb[p], lo = row < j ? row : j, hi = row < j ? j : row;
                    int sid[L];
#pragma unroll
                    for (int c = 0; c < L; ++c) sid[c] = sm.nb[P_[c]];
                    if (take_edge(P.adj, W, lo, hi)) {
                        atomicAdd(reinterpret_cast<unsigned long long *>(&sm.removed), 1ull);
                        write_record(P, lo, hi, L, sid);
                    }
                }
            }
        }
        if (my_tests) atomicAdd(reinterpret_cast<unsigned long long *>(&sm.tests), (unsigned long long)my_tests);
        __syncthreads();
        // Settle the staged independent tests: one winner per edge, consecutive SepSet slots.
        const int nst = sm.nstage < kProbeStage ? sm.nstage : kProbeStage;
        if (nst > 0) {
            int myslot = -1, e = 0;
            if (tid < nst) {
                e = sm.stage[tid];
                const int j = sm.nb[e / nsub], lo = row < j ? row : j, hi = row < j ? j : row;
                if (take_edge(P.adj, W, lo, hi)) myslot = atomicAdd(&sm.nwin, 1);
            }
            __syncthreads();
            if (tid == 0) {
                const int nw = sm.nwin;
                sm.rec_base = nw ? atomicAdd(reinterpret_cast<unsigned long long *>(P.rec_count), (unsigned long long)nw)
                                 : 0ull;
                sm.removed += nw;
            }
            __syncthreads();
            if (myslot >= 0) {
                const long long k = (long long)(sm.rec_base + (unsigned long long)myslot);
                if (k < P.rec_cap) {
                    const int p = e / nsub, j = sm.nb[p];
                    int P_[L], sid[L];
                    subset(p, e - p * nsub, P_);
#pragma unroll
                    for (int c = 0; c < L; ++c) sid[c] = sm.nb[P_[c]];
                    store_record(P.recs + k, row < j ? row : j, row < j ? j : row, L, sid);
                }
            }
            if (tid == 0) {
                sm.nstage = 0;
                sm.nwin = 0;
            }
        }
    }
    __syncthreads();
    if (tid == 0 && stats_pd >= 0) {
        Prob &Ps = b.probs[stats_pd];
        if (sm.tests) { add_ll(&Ps.tests[L], sm.tests); add_ll(&Ps.probe_tests[L], sm.tests); }
        if (sm.removed) { add_ll(&Ps.removed[L], sm.removed); add_ll(&Ps.probe_removed[L], sm.removed); }
    }
}

// ---------------------------------------------------------------------------------------------
// Row order: the MLP ranks the candidates k of every node i (the shared-set form of the ordering)
// ---------------------------------------------------------------------------------------------
// A conditioning set of the level kernel serves every edge of its row (the set sharing of cuPC-S,
// Sec. 3.4), so the unit the model ranks here is the candidate k of node i. Its features, all
// from quantities the method computes (C and G' at the start of the level):
//   |C_ik|, |C_ik| / max_q |C_iq|, min(n |N_i & N_k| / (d_i d_k), 8) / 8, d_k / (d_i + d_k),
//   |C_k k*| and |rho_ik.k*| (k* the candidate of largest |C_ik|; 1 and 0 for k = k*),
//   mean_j |C_ij| / max_q |C_iq|, |N_i & N_k| / d_i.
// The fifth and sixth tell the model how much a candidate adds to k*, which the order always tests
// first; the model picks the others.
constexpr int kRowCap = kRowOrderCap;      // rows up to this degree are ranked (neighbour list in LDS)
constexpr int kRowWords = kRowOrderWords;  // adjacency words of a row staged in LDS (n <= 16384)
constexpr int kRowTopMax = 16;
constexpr int kRowShortMax = 64;   // longest short list the model scores (one tile per wavefront)

template <typename T>
struct __align__(16) RowSmem {
    uint16_t W1[kHid][8];
    uint16_t W2[kHid][kHid + 8];
    uint16_t X[4][64][8];
    uint16_t H1[4][16][kHid + 8];
    int nb[kRowCap];
    float ac[kRowCap];     // |C_ik| (entries past d hold -1, so rank counts can read in fours)
    float sc[kRowCap];     // MLP score (entries past d hold -inf)
    T ci[kRowCap];         // C_ik
    unsigned long long arow[kRowWords];
    float b1[kHid], b2[kHid], W3[kHid];
    int toppos[kRowTopMax];
    int stage[kProbeStage];    // (top index, position) of the independent tests of the row
    int nstage, nwin;
    unsigned long long rec_base;
    long long tests, removed;
    float red[4], redmax[4];
    float b3;
    alignas(16) int taken[kRowCap];   // candidate chosen (argmax rounds); separated-by-k* flags
    int kstar;             // position of the candidate of largest |C_ik| (lowest position on ties)
    int slist[kRowShortMax];     // short list: positions of the largest |C_ik|, in that order
    float sshort[kRowShortMax];  // model scores of the short list
    int scn[kRowShortMax];       // |N_i & N_k| of the short list
    int sel_n, tie_n, sel_b, sel_above;   // short-list selection: counts, bucket B, members before B
    float bestv[4];
    int besti[4];
};

// Loads the MLP parameters into LDS (BF16 weights, FP32 biases).
template <class Smem>
__device__ inline void load_mlp_bf16(Smem &sm, const float *params, int tid, int nthreads) {
    // The parameters come through a generic pointer, which the compiler cannot tell apart from
    // LDS: a load-convert-store loop would wait for every load before its store. With 256 threads
    // every value a thread needs is loaded first (W2: 16 consecutive values, W1: 2), then stored.
    if (nthreads == kHid * kHid / 16) {
        float w2[16], w1[2], bb[3] = {0.f, 0.f, 0.f}, b3 = 0.f;
#pragma unroll
        for (int u = 0; u < 16; ++u) w2[u] = params[oW2 + 16 * tid + u];
#pragma unroll
        for (int u = 0; u < 2; ++u) w1[u] = params[oW1 + 2 * tid + u];
        if (tid < kHid) {
            bb[0] = params[oB1 + tid];
            bb[1] = params[oB2 + tid];
            bb[2] = params[oW3 + tid];
        }
        if (tid == 0) b3 = params[oB3];
#pragma unroll
        for (int u = 0; u < 16; ++u) sm.W2[(16 * tid + u) / kHid][(16 * tid + u) % kHid] = bf16_rne(w2[u]);
#pragma unroll
        for (int u = 0; u < 2; ++u) sm.W1[(2 * tid + u) / kIn][(2 * tid + u) % kIn] = bf16_rne(w1[u]);
        if (tid < kHid) {
            sm.b1[tid] = bb[0];
            sm.b2[tid] = bb[1];
            sm.W3[tid] = bb[2];
        }
        if (tid == 0) sm.b3 = b3;
        return;
    }
    for (int e = tid; e < kHid * kIn; e += nthreads) sm.W1[e / kIn][e % kIn] = bf16_rne(params[oW1 + e]);
    for (int e = tid; e < kHid * kHid; e += nthreads) sm.W2[e / kHid][e % kHid] = bf16_rne(params[oW2 + e]);
    if (tid < kHid) {
        sm.b1[tid] = params[oB1 + tid];
        sm.b2[tid] = params[oB2 + tid];
        sm.W3[tid] = params[oW3 + tid];
    }
    if (tid == 0) sm.b3 = params[oB3];
}

// Scores the 64 feature rows in sm.X[wave] (BF16) with the MLP; writes rows r < nrows of them to
// out[r - r0] for r = r0 .. r0 + 63 (one wavefront).
template <class Smem>
__device__ inline void mlp_score64(Smem &sm, int wave, int lane, int r0, int nrows, float *out) {
    const bf16x8 zero8 = {};
    const int tiles = (nrows - r0 + 15) / 16 < 4 ? (nrows - r0 + 15) / 16 : 4;
    for (int mt = 0; mt < tiles; ++mt) {
        const bf16x8 ax = lane < 16 ? *reinterpret_cast<const bf16x8 *>(&sm.X[wave][16 * mt + lane][0]) : zero8;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const bf16x8 bw = lane < 16 ? *reinterpret_cast<const bf16x8 *>(&sm.W1[16 * nt + lane][0]) : zero8;
            const floatx4 z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, bw, floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            const int col = 16 * nt + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float h = z[v] + sm.b1[col];
                sm.H1[wave][4 * (lane >> 4) + v][col] = bf16_rne(h > 0.0f ? h : 0.0f);
            }
        }
        wave_sync_lds();
        floatx4 acc[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const bf16x8 ah = *reinterpret_cast<const bf16x8 *>(&sm.H1[wave][lane & 15][32 * ks + 8 * (lane >> 4)]);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const bf16x8 bw = *reinterpret_cast<const bf16x8 *>(&sm.W2[16 * nt + (lane & 15)][32 * ks + 8 * (lane >> 4)]);
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bw, acc[nt], 0, 0, 0);
            }
        }
        wave_sync_lds();
        float part[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float sacc = 0.0f;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const int col = 16 * nt + (lane & 15);
                const float h = acc[nt][v] + sm.b2[col];
                sacc += (h > 0.0f ? h : 0.0f) * sm.W3[col];
            }
            part[v] = sacc;
        }
#pragma unroll
        for (int o = 1; o < 16; o <<= 1)
#pragma unroll
            for (int v = 0; v < 4; ++v) part[v] += __shfl_xor(part[v], o, 64);
        if ((lane & 15) == 0)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = r0 + 16 * mt + 4 * (lane >> 4) + v;
                if (r < nrows) out[r - r0] = part[v] + sm.b3;
            }
    }
}

// Stages row i (neighbours, |C_ik|, its adjacency words) and returns the row mean of |C_ik|.
template <typename T, class Smem>
__device__ inline float stage_row(Smem &sm, const Prob &P, int row, int d, int tid, int nthreads, float &rowmax) {
    const int64_t n = P.n, W = P.W;
    const T *C = static_cast<const T *>(P.C);
    float s = 0.0f;
    for (int p = tid; p < d; p += nthreads) {
        const int k = P.nbr[(int64_t)row * n + p];
        sm.nb[p] = k;
        const T c = C[(int64_t)row * n + k];
        sm.ci[p] = c;
        const float a = fabsf((float)c);
        sm.ac[p] = a;
        s += a;
    }
    for (int p = d + tid; p < ((d + 3) & ~3); p += nthreads) sm.ac[p] = -1.0f;
    for (int w = tid; w < W && w < kRowWords; w += nthreads) sm.arow[w] = P.adj[(int64_t)row * W + w];
    // The largest |C_ik| and its lowest position.
    float mx = -1.0f;
    int mp = 0x7fffffff;
    for (int p = tid; p < d; p += nthreads)
        if (sm.ac[p] > mx) {   // ascending p per thread: the first maximum is kept
            mx = sm.ac[p];
            mp = p;
        }
    for (int o = 32; o >= 1; o >>= 1) {
        s += __shfl_xor(s, o, 64);
        const float om = __shfl_xor(mx, o, 64);
        const int op = __shfl_xor(mp, o, 64);
        if (om > mx || (om == mx && op < mp)) { mx = om; mp = op; }
    }
    if ((tid & 63) == 0) {
        sm.red[tid >> 6] = s;
        sm.redmax[tid >> 6] = mx;
        sm.besti[tid >> 6] = mp;
    }
    __syncthreads();
    float bm = sm.redmax[0];
    int bp = sm.besti[0];
    for (int w = 1; w < 4; ++w)
        if (sm.redmax[w] > bm || (sm.redmax[w] == bm && sm.besti[w] < bp)) { bm = sm.redmax[w]; bp = sm.besti[w]; }
    rowmax = bm > 0.0f ? bm : 0.0f;
    if (tid == 0) sm.kstar = bp;
    __syncthreads();
    return ((sm.red[0] + sm.red[1]) + (sm.red[2] + sm.red[3])) / (float)d;
}

// Features of candidate position p of the staged row (see above). All of them are ratios or
// correlations, so that a model trained on small graphs carries over to larger, sparser ones.
template <typename T, class Smem>
__device__ inline void row_features(const Smem &sm, const Prob &P, int d, int p, int level, float rowmean,
                                    float rowmax, float (&x)[kIn], int cn_given = -1) {
    (void)level;
    const int64_t W = P.W;
    const T *C = static_cast<const T *>(P.C);
    const float a = sm.ac[p];
    const int k = sm.nb[p];
    const int ps = sm.kstar, ks = sm.nb[ps];
    // C_k k*, and the partial correlation of i and k given k* (zero for k* itself)
    const float ckk = p == ps ? 1.0f : (float)C[(int64_t)ks * P.n + k];
    float rho = 0.0f;
    if (p != ps) {
        const float cik = (float)sm.ci[p], cis = (float)sm.ci[ps];
        const float den = (1.0f - cis * cis) * (1.0f - ckk * ckk);
        rho = den > 0.0f ? fminf(1.0f, fabsf(cik - cis * ckk) * __builtin_amdgcn_rsqf(den)) : 0.0f;
    }
    // G is not written while the order is computed (before the level's tests), so plain loads.
    int cn = cn_given;   // |N_i & N_k| (the caller guarantees W <= kRowWords)
    if (cn < 0) {
        const unsigned long long *ak = P.adj + (int64_t)k * W;
        cn = 0;
#pragma unroll 8
        for (int64_t w = 0; w < W; ++w) cn += __popcll(sm.arow[w] & ak[w]);
    }
    const float di = (float)d, dk = (float)P.deg[k];
    // overlap against a random graph of the same degrees: n |N_i & N_k| / (d_i d_k)
    const float lift = dk > 0.0f ? (float)cn * (float)P.n / (di * dk) : 0.0f;
    x[0] = a;
    x[1] = rowmax > 0.0f ? a / rowmax : 0.0f;
    x[2] = fminf(lift, 8.0f) / 8.0f;
    x[3] = dk / (di + dk);
    x[4] = fabsf(ckk);
    x[5] = rho;
    x[6] = rowmax > 0.0f ? rowmean / rowmax : 0.0f;
    x[7] = (float)cn / di;
}

// One work-group per row of G' at level 1 (grid-stride), the first part of the level with the
// shared-set order:
//  1. rows with 2 <= d <= kRowCap (and n <= 64 kRowWords): the MLP scores every candidate k of the
//     row (features staged in LDS), and the row's neighbour list is rewritten with the `top`
//     best-scored candidates first (best first; the others keep their ascending order);
//  2. every row with d >= 2: the sets {k} of its first `top` positions (the best-scored, or simply
//     the first for rows too long to score) are tested against every live edge (i, j) of the row
//     with the level's FP32 test (same band and re-check queue). Independent tests are staged and
//     settled together (one winner per edge, one SepSet slot reservation per row).
// The rest of the level then runs over the ranks top .. d - 1 of the rewritten lists.
template <typename T>
// With scores_out (n x n, problem 0 only) the kernel only ranks: it writes each scored candidate's
// score at [i][k] (-inf for candidates outside the short list) and the chosen candidates at
// top_out[i][0 .. top) (best first, -1 past the row's choices), and runs no test.
__global__ __launch_bounds__(256, 4) void k_row_order(Batch b, int level, const float *params, int top, int by_abs,
                                                    int short_k, int sort_rest, float *scores_out, int *top_out) {
    __shared__ RowSmem<T> sm;
    if (b.st->done) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (!by_abs) load_mlp_bf16(sm, params, tid, 256);
    if (tid == 0) {
        sm.tests = 0;
        sm.removed = 0;
        sm.nstage = 0;
        sm.nwin = 0;
    }
    int stats_pd = -1;
    for (long long grow = blockIdx.x; grow < b.total_rows; grow += gridDim.x) {
        const int pd = find_base(b.row_base, b.count, grow);
        Prob &P = b.probs[pd];
        const int row = (int)(grow - b.row_base[pd]);
        const int d = P.deg[row];
        if (d < 2 || !(level <= P.max_level && P.tau[level] == P.tau[level])) continue;
        __syncthreads();   // the previous row's LDS contents and statistics are no longer read
        if (tid == 0 && pd != stats_pd) {
            if (stats_pd >= 0) {
                Prob &Ps = b.probs[stats_pd];
                if (sm.tests) { add_ll(&Ps.tests[level], sm.tests); add_ll(&Ps.probe_tests[level], sm.tests); }
                if (sm.removed) {
                    add_ll(&Ps.removed[level], sm.removed);
                    add_ll(&Ps.probe_removed[level], sm.removed);
                }
            }
            sm.tests = 0;
            sm.removed = 0;
        }
        stats_pd = pd;
        const int64_t n = P.n, W = P.W;
        const T *C = static_cast<const T *>(P.C);
        int *nbr = P.nbr + (int64_t)row * n;
        const bool scored = l1_ranked(d, W);
        const int T_ = top < d ? top : d;
        if (scored) {
            float rowmax = 0.0f;
            const float rowmean = stage_row<T>(sm, P, row, d, tid, 256, rowmax);
            if (by_abs) {
                // |C_ik| alone ranks the candidates (no model).
                for (int p = tid; p < d; p += 256) sm.sc[p] = sm.ac[p];
            } else if (short_k > 0 && d > short_k) {
                // Only the short_k candidates of largest |C_ik| (ties: lower position) are scored by
                // the model; the others cannot be chosen. slist[r] is the candidate of place r in that
                // order. A histogram of |C_ik| in 256 buckets (largest first) gives the bucket B that
                // holds the short_k-th candidate: the buckets before it are all in, and only B's few
                // members are ranked exactly.
                int *hist = sm.stage;            // free until the tests
                int *tie = sm.taken;             // free until the argmax rounds
                hist[tid] = 0;
                if (tid == 0) { sm.sel_n = 0; sm.tie_n = 0; }
                __syncthreads();
                int bk[kRowCap / 256];
#pragma unroll
                for (int c = 0; c < kRowCap / 256; ++c) {
                    const int p = tid + 256 * c;
                    bk[c] = -1;
                    if (p < d) {
                        const int key = (int)(sm.ac[p] * 256.0f);
                        bk[c] = 255 - (key < 0 ? 0 : (key > 255 ? 255 : key));
                        atomicAdd(&hist[bk[c]], 1);
                    }
                }
                __syncthreads();
                if (tid < 64) {   // exclusive scan of the buckets, four per lane; B and the count before it
                    int v[4], tot = 0;
#pragma unroll
                    for (int c = 0; c < 4; ++c) { v[c] = hist[4 * tid + c]; tot += v[c]; }
                    int incl = tot;
#pragma unroll
                    for (int o = 1; o < 64; o <<= 1) {
                        const int t = __shfl_up(incl, o, 64);
                        if (tid >= o) incl += t;
                    }
                    int run = incl - tot;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        if (run < short_k && run + v[c] >= short_k) { sm.sel_b = 4 * tid + c; sm.sel_above = run; }
                        run += v[c];
                    }
                }
                __syncthreads();
                const int B = sm.sel_b;
#pragma unroll
                for (int c = 0; c < kRowCap / 256; ++c) {
                    const int p = tid + 256 * c;
                    if (bk[c] >= 0 && bk[c] < B) sm.slist[atomicAdd(&sm.sel_n, 1)] = p;
                    else if (bk[c] == B) tie[atomicAdd(&sm.tie_n, 1)] = p;
                }
                __syncthreads();
                // B's members by place (|C_ik| descending, then position); the first short_k - above
                // of them complete the list
                const int above = sm.sel_above, nt = sm.tie_n;
                for (int t = tid; t < nt; t += 256) {
                    const int p = tie[t];
                    const float a = sm.ac[p];
                    int r = 0;
                    for (int u = 0; u < nt; ++u) {
                        const int q = tie[u];
                        const float aq = sm.ac[q];
                        r += (aq > a || (aq == a && q < p)) ? 1 : 0;
                    }
                    if (r < short_k - above) sm.slist[above + r] = p;
                }
                __syncthreads();
                // places among the chosen short_k (they are all in slist, unordered before `above`)
                {
                    int p = -1, r = 0;
                    if (tid < short_k) {
                        p = sm.slist[tid];
                        const float a = sm.ac[p];
                        for (int u = 0; u < short_k; ++u) {
                            const int q = sm.slist[u];
                            const float aq = sm.ac[q];
                            r += (aq > a || (aq == a && q < p)) ? 1 : 0;
                        }
                    }
                    __syncthreads();
                    if (tid < short_k) sm.slist[r] = p;
                }
                for (int p = tid; p < d; p += 256) sm.sc[p] = -INFINITY;
                // |N_i & N_k| of the short list, all threads at once: one (candidate, word) pair
                // each, so the adjacency rows of the K candidates are read in one round.
                if (tid < short_k) sm.scn[tid] = 0;
                __syncthreads();
                for (int e = tid; e < short_k * (int)W; e += 256) {
                    const int r = e / (int)W, w = e - r * (int)W;
                    const int c = __popcll(sm.arow[w] & P.adj[(int64_t)sm.nb[sm.slist[r]] * W + w]);
                    if (c) atomicAdd(&sm.scn[r], c);
                }
                __syncthreads();
                for (int r0 = 64 * wave; r0 < short_k; r0 += 256) {
                    float x[kIn] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                    if (r0 + lane < short_k)
                        row_features<T>(sm, P, d, sm.slist[r0 + lane], level, rowmean, rowmax, x, sm.scn[r0 + lane]);
#pragma unroll
                    for (int u = 0; u < kIn; ++u) sm.X[wave][lane][u] = bf16_rne(x[u]);
                    wave_sync_lds();
                    mlp_score64(sm, wave, lane, r0, short_k, sm.sshort + r0);
                    wave_sync_lds();
                    if (r0 + lane < short_k) sm.sc[sm.slist[r0 + lane]] = sm.sshort[r0 + lane];
                }
            } else {
                for (int r0 = 64 * wave; r0 < d; r0 += 256) {
                    float x[kIn] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                    if (r0 + lane < d) row_features<T>(sm, P, d, r0 + lane, level, rowmean, rowmax, x);
#pragma unroll
                    for (int u = 0; u < kIn; ++u) sm.X[wave][lane][u] = bf16_rne(x[u]);
                    wave_sync_lds();
                    mlp_score64(sm, wave, lane, r0, d, sm.sc + r0);
                    wave_sync_lds();
                }
            }
            for (int p = d + tid; p < ((d + 3) & ~3); p += 256) sm.sc[p] = -INFINITY;
            __syncthreads();
            // The model picks the candidates after k* (largest |C_ik|), which always comes first
            // (written once every wavefront's scores are in).
            if (!by_abs) {
                if (tid == 0) sm.sc[sm.kstar] = INFINITY;
                __syncthreads();
            }
            // The top T_ by score: T_ rounds of a work-group argmax (ties: lower position first).
            for (int p = tid; p < d; p += 256) sm.taken[p] = 0;
            __syncthreads();
            for (int u = 0; u < T_; ++u) {
                float bv = -INFINITY;
                int bi = 0x7fffffff;
                for (int p = tid; p < d; p += 256)
                    if (!sm.taken[p] && (sm.sc[p] > bv || (sm.sc[p] == bv && p < bi))) {
                        bv = sm.sc[p];
                        bi = p;
                    }
                for (int o = 32; o >= 1; o >>= 1) {
                    const float ov = __shfl_xor(bv, o, 64);
                    const int oi = __shfl_xor(bi, o, 64);
                    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
                }
                if (lane == 0) {
                    sm.bestv[wave] = bv;
                    sm.besti[wave] = bi;
                }
                __syncthreads();
                if (tid == 0) {
                    float v = sm.bestv[0];
                    int i = sm.besti[0];
                    for (int w = 1; w < 4; ++w)
                        if (sm.bestv[w] > v || (sm.bestv[w] == v && sm.besti[w] < i)) { v = sm.bestv[w]; i = sm.besti[w]; }
                    sm.toppos[u] = i;
                    sm.taken[i] = 1;
                }
                __syncthreads();
            }
            if (scores_out) {
                for (int p = tid; p < d; p += 256) scores_out[(int64_t)row * n + sm.nb[p]] = sm.sc[p];
                if (tid < top) top_out[(int64_t)row * top + tid] = tid < T_ ? sm.nb[sm.toppos[tid]] : -1;
                continue;
            }
            if (sort_rest && 2 * (int64_t)d <= n) {
                // Sorted enumeration: the list stays ascending (the level kernel's lanes then read
                // ascending columns of C), and the set order goes after it as a permutation of
                // positions: the chosen candidates, then the others by descending |C_ik| in 256
                // buckets (a counting sort; the order inside a bucket is that of the LDS atomics,
                // which only changes which separating set a level finds first).
                int *cnt = sm.stage;    // bucket counters, then offsets (free until the tests)
                cnt[tid] = 0;
                __syncthreads();
                int mine[4], slot[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int p = tid + 256 * c;
                    mine[c] = -1;
                    if (p < d && !sm.taken[p]) {
                        const int key = (int)(sm.ac[p] * 255.99f);
                        mine[c] = 255 - (key < 0 ? 0 : (key > 255 ? 255 : key));
                        slot[c] = atomicAdd(&cnt[mine[c]], 1);
                    }
                }
                __syncthreads();
                if (tid < 64) {   // exclusive scan of the 256 counters, four per lane
                    int v[4], tot = 0;
#pragma unroll
                    for (int c = 0; c < 4; ++c) { v[c] = cnt[4 * tid + c]; tot += v[c]; }
                    int incl = tot;
#pragma unroll
                    for (int o = 1; o < 64; o <<= 1) {
                        const int t = __shfl_up(incl, o, 64);
                        if (tid >= o) incl += t;
                    }
                    int run = incl - tot;
#pragma unroll
                    for (int c = 0; c < 4; ++c) { cnt[4 * tid + c] = run; run += v[c]; }
                }
                __syncthreads();
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (mine[c] >= 0) nbr[d + T_ + cnt[mine[c]] + slot[c]] = tid + 256 * c;
                if (tid < T_) nbr[d + tid] = sm.toppos[tid];
                __syncthreads();   // the counters' storage is the tests' staging area
            } else {
                // New order: the top candidates by rank, then the others in their (ascending) order.
                for (int p = tid; p < d; p += 256) {
                    int pos = -1, below = 0;
                    for (int u = 0; u < T_; ++u) {
                        const int tp = sm.toppos[u];
                        if (tp == p) pos = u;
                        below += tp < p ? 1 : 0;
                    }
                    nbr[pos >= 0 ? pos : T_ + p - below] = sm.nb[p];
                }
            }
        } else if (tid < T_) {
            sm.toppos[tid] = tid;   // too long to score: the first positions, order unchanged
        }
        if (scores_out) {
            if (!scored && tid < top) top_out[(int64_t)row * top + tid] = tid < T_ ? nbr[tid] : -1;
            continue;
        }
        __syncthreads();
        // 2. The sets {k} of the top candidates against every live edge of the row.
        auto NB = [&](int q) -> int { return scored ? sm.nb[q] : nbr[q]; };
        auto CIv = [&](int q) -> T { return scored ? sm.ci[q] : C[(int64_t)row * n + nbr[q]]; };
        auto LIVE = [&](int j) -> bool {
            const unsigned long long wv = scored ? sm.arow[j >> 6] : live_word(P.adj + (int64_t)row * W + (j >> 6));
            return (wv >> (j & 63)) & 1ull;
        };
        const double tau = P.tau[level];
        const float tl = P.t[level], band = P.band[level];
        long long my_tests = 0;
        for (int e = tid; e < T_ * d; e += 256) {
            const int u = e / d, q = e - u * d, kp = sm.toppos[u];
            if (q == kp) continue;
            const int j = NB(q);
            if (!LIVE(j)) continue;
            const int k = NB(kp);
            const int P1[1] = {kp};
            auto CS1 = [&](int a, int c) -> T { return (T)1; };   // only the diagonal of M2 = [1]
            auto CI1 = [&](int a) -> T { return CIv(a); };
            SetFactor<T, 1> f;
            f.build(P1, CS1, CI1);
            // C[k, j] from the row of the set element (C is exactly symmetric): the threads of a set
            // read ascending columns of one row instead of one row each
            const T col[1] = {C[(int64_t)k * n + j]};
            ++my_tests;
            const int dec = f.test_vals(col, CIv(q), tau, tl, band);
            if (dec == 2) {
                const int sid[1] = {k};
                push_recheck<1>(b, pd, row, j, sid, 2);
            } else if (dec == 1) {
                const int slot = atomicAdd(&sm.nstage, 1);
                if (slot < kProbeStage) {
                    sm.stage[slot] = e;
                } else {
                    const int lo = row < j ? row : j, hi = row < j ? j : row;
                    const int sid[1] = {k};
                    if (take_edge(P.adj, W, lo, hi)) {
                        atomicAdd(reinterpret_cast<unsigned long long *>(&sm.removed), 1ull);
                        write_record(P, lo, hi, 1, sid);
                    }
                }
            }
        }
        if (my_tests) atomicAdd(reinterpret_cast<unsigned long long *>(&sm.tests), (unsigned long long)my_tests);
        __syncthreads();
        // Settle the staged independent tests: one winner per edge, consecutive SepSet slots.
        const int nst = sm.nstage < kProbeStage ? sm.nstage : kProbeStage;
        if (nst > 0) {
            int myslot = -1, e = 0;
            if (tid < nst) {
                e = sm.stage[tid];
                const int j = NB(e % d), lo = row < j ? row : j, hi = row < j ? j : row;
                if (take_edge(P.adj, W, lo, hi)) myslot = atomicAdd(&sm.nwin, 1);
            }
            __syncthreads();
            if (tid == 0) {
                const int nw = sm.nwin;
                sm.rec_base = nw ? atomicAdd(reinterpret_cast<unsigned long long *>(P.rec_count), (unsigned long long)nw)
                                 : 0ull;
                sm.removed += nw;
            }
            __syncthreads();
            if (myslot >= 0) {
                const long long kk = (long long)(sm.rec_base + (unsigned long long)myslot);
                if (kk < P.rec_cap) {
                    const int j = NB(e % d), sid[1] = {NB(sm.toppos[e / d])};
                    store_record(P.recs + kk, row < j ? row : j, row < j ? j : row, 1, sid);
                }
            }
            if (tid == 0) {
                sm.nstage = 0;
                sm.nwin = 0;
            }
        }
    }
    __syncthreads();
    if (tid == 0 && stats_pd >= 0) {
        Prob &Ps = b.probs[stats_pd];
        if (sm.tests) { add_ll(&Ps.tests[level], sm.tests); add_ll(&Ps.probe_tests[level], sm.tests); }
        if (sm.removed) { add_ll(&Ps.removed[level], sm.removed); add_ll(&Ps.probe_removed[level], sm.removed); }
    }
}

// Training rows of the shared-set order at level 1: the features of every candidate k of every
// node i, and a label from the FP32 test |rho_ij.k| <= tanh(tau_1) (Eq. 3-6 at l = 1, without the
// re-check band) over the other edges (i, j), j in N_i \ {k}: for k*, the candidate of largest
// |C_ik|, the fraction of them that {k*} separates; for every other k, the fraction that {k}
// separates and {k*} does not. The model thus ranks k* by what it removes and the others by what
// they add to it, which is what the second and later choices are worth. meta gets (i, k).
template <typename T>
__global__ __launch_bounds__(256) void k_row_features(Batch b, int level, const long long *foff, float *feats,
                                                      float *labels, int *meta, const int *skip) {
    __shared__ RowSmem<T> sm;
    if (*skip) return;
    const int tid = threadIdx.x;
    const long long grow = blockIdx.x;
    const int pd = find_base(b.row_base, b.count, grow);
    const Prob &P = b.probs[pd];
    const int row = (int)(grow - b.row_base[pd]);
    const int d = P.deg[row];
    if (d < 1 || d > kRowCap || P.W > kRowWords) return;
    float rowmax = 0.0f;
    const float rowmean = stage_row<T>(sm, P, row, d, tid, 256, rowmax);
    const int64_t n = P.n;
    const T *C = static_cast<const T *>(P.C);
    const float tl = (float)tanh(P.tau[1]);
    const long long base = foff[grow];
    auto separates = [&](int q, int k, float cik) -> bool {   // {k} separates (i, N_i[q])
        const int j = sm.nb[q];
        const float cij = (float)C[(int64_t)row * n + j], cjk = (float)C[(int64_t)j * n + k];
        const float den = (1.0f - cik * cik) * (1.0f - cjk * cjk);
        return den > 0.0f && fabsf(cij - cik * cjk) <= tl * sqrtf(den);
    };
    const int ps = sm.kstar, kst = sm.nb[ps];
    const float cist = (float)C[(int64_t)row * n + kst];
    for (int q = tid; q < d; q += 256) sm.taken[q] = q != ps && separates(q, kst, cist) ? 1 : 0;
    __syncthreads();
    for (int p = tid; p < d; p += 256) {
        float x[kIn];
        row_features<T>(sm, P, d, p, level, rowmean, rowmax, x);
        float *f = feats + (base + p) * kIn;
#pragma unroll
        for (int u = 0; u < kIn; ++u) f[u] = x[u];
        const int k = sm.nb[p];
        const float cik = (float)C[(int64_t)row * n + k];
        int sep = 0;
        for (int q = 0; q < d; ++q) {
            if (q == p) continue;
            if (p != ps && sm.taken[q]) continue;   // already separated by k*
            sep += separates(q, k, cik) ? 1 : 0;
        }
        labels[base + p] = d > 1 ? (float)sep / (float)(d - 1) : 0.0f;
        if (meta) {
            meta[(base + p) * 2 + 0] = row;
            meta[(base + p) * 2 + 1] = k;
        }
    }
}

// grid: compute units; as many work-groups per unit as fit are launched.
template <typename T>
static hipError_t launch_row_order_t(hipStream_t s, const Batch &b, int level, const float *params, int top,
                                     int by_abs, int short_k, int sort_rest, int grid, float *scores_out,
                                     int *top_out) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_row_order<T>, 256, 0) != hipSuccess || per_cu < 1)
        per_cu = 2;
    hipLaunchKernelGGL(k_row_order<T>, dim3(per_cu * grid), dim3(256), 0, s, b, level, params, top, by_abs, short_k,
                       sort_rest, scores_out, top_out);
    return hipGetLastError();
}

hipError_t launch_row_order(hipStream_t s, const Batch &b, int level, const float *params, int top, int by_abs,
                            int short_k, int sort_rest, int grid, float *scores_out, int *top_out) {
    if (top < 1 || top > kRowTopMax || short_k < 0 || short_k > kRowShortMax) return hipErrorInvalidValue;
    if (!by_abs && !params) return hipErrorInvalidValue;
    if ((scores_out != nullptr) != (top_out != nullptr) || (scores_out && b.count != 1)) return hipErrorInvalidValue;
    if (b.prec == PC_PREC_FP64)
        return launch_row_order_t<double>(s, b, level, params, top, by_abs, short_k, sort_rest, grid, scores_out,
                                          top_out);
    return launch_row_order_t<float>(s, b, level, params, top, by_abs, short_k, sort_rest, grid, scores_out, top_out);
}

hipError_t launch_row_features(hipStream_t s, const Batch &b, int level, long long *foff, long long cap, int *skip,
                               float *feats, float *labels, int *meta) {
    hipLaunchKernelGGL(k_feat_plan, dim3(1), dim3(1024), 0, s, b, foff, cap, skip, 1);
    if (b.prec == PC_PREC_FP64)
        hipLaunchKernelGGL(k_row_features<double>, dim3((unsigned)b.total_rows), dim3(256), 0, s, b, level, foff, feats,
                           labels, meta, skip);
    else
        hipLaunchKernelGGL(k_row_features<float>, dim3((unsigned)b.total_rows), dim3(256), 0, s, b, level, foff, feats,
                           labels, meta, skip);
    return hipGetLastError();
}

template <typename T, int L>
struct ProbeDispatch {
    static hipError_t run(hipStream_t s, const Batch &b, int level, const float *params, int topq, int grid) {
        if (level == L) {
            // As many work-groups as fit at once (each keeps its row's block and scores in LDS).
            int per_cu = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_probe<T, L>, kProbeThreads, 0) == hipSuccess &&
                per_cu > 0)
                grid = per_cu * grid;
            hipLaunchKernelGGL((k_probe<T, L>), dim3(grid), dim3(kProbeThreads), 0, s, b, params, topq);
            return hipGetLastError();
        }
        return ProbeDispatch<T, L + 1>::run(s, b, level, params, topq, grid);
    }
};
template <typename T>
struct ProbeDispatch<T, kTopMax + 1> {
    static hipError_t run(hipStream_t, const Batch &, int, const float *, int, int) { return hipErrorInvalidValue; }
};

hipError_t launch_probe(hipStream_t s, const Batch &b, int level, const float *params, int topq, int grid) {
    if (level < 1 || level > kTopMax || topq < 1 || topq > kTopMax) return hipErrorInvalidValue;
    if (b.prec == PC_PREC_FP64) return ProbeDispatch<double, 1>::run(s, b, level, params, topq, grid);
    return ProbeDispatch<float, 1>::run(s, b, level, params, topq, grid);
}

}  // namespace pcg
