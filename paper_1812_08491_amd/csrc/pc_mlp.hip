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
__global__ __launch_bounds__(1024) void k_feat_plan(Batch b, long long *foff, long long cap, int *skip) {
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
        return dg * (dg - 1);
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

// ---------------------------------------------------------------------------------------------
// Probe: per directed edge, the subsets of its top-Q candidates
// ---------------------------------------------------------------------------------------------
constexpr int kTopMax = 8;

struct SmallBinom {
    __device__ unsigned long long operator()(int a, int b) const {
        if (b < 0 || a < b) return 0ull;
        unsigned long long c = 1;
        for (int k = 0; k < b; ++k) c = c * (unsigned long long)(a - k) / (unsigned long long)(k + 1);
        return c;
    }
};

// One work-group per flattened row i; wave w takes the edges (i, N_i[p]) with p = w (mod 4).
template <typename T, int L>
__global__ __launch_bounds__(256) void k_probe(Batch b, const long long *foff, const float *scores,
                                               int topq, const int *skip) {
    __shared__ long long s_tests, s_removed;
    if (*skip) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) { s_tests = 0; s_removed = 0; }
    __syncthreads();
    const long long grow = blockIdx.x;
    const int pd = find_base(b.row_base, b.count, grow);
    const Prob &P = b.probs[pd];
    const int64_t n = P.n, W = P.W;
    const int row = (int)(grow - b.row_base[pd]);
    const int d = P.deg[row];
    long long my_tests = 0, my_removed = 0;
    if (d >= L + 1 && L <= P.max_level && P.tau[L] == P.tau[L]) {
        const T *C = static_cast<const T *>(P.C);
        const int *nb = P.nbr + (int64_t)row * n;
        unsigned long long *adj_row = P.adj + (int64_t)row * W;
        auto CS = [&](int p, int q) -> T { return p == q ? (T)1 : C[(int64_t)nb[p] * n + nb[q]]; };
        auto CI = [&](int p) -> T { return C[(int64_t)row * n + nb[p]]; };
        const double tau = P.tau[L];
        const float tl = P.t[L], band = P.band[L];
        const int Q = d - 1 <= 64 * 64 ? min(min(topq, kTopMax), d - 1) : 0;  // 64-bit taken mask
        const unsigned long long nsub = SmallBinom()(Q, L);
        for (int p = wave; p < d; p += 4) {
            const int j = nb[p];
            if (!((live_word(adj_row + (j >> 6)) >> (j & 63)) & 1ull)) continue;
            // Top-Q candidates by score (ties: lower position first), by Q rounds of wave argmax.
            const float *sc = scores + foff[grow] + (long long)p * (d - 1);
            unsigned long long taken = 0ull;  // this lane's entries qq = lane + 64 t already chosen
            int top[kTopMax];
#pragma unroll
            for (int u = 0; u < kTopMax; ++u) {
                top[u] = -1;
                if (u >= Q) continue;
                float best = -INFINITY;
                int bi = 0x7fffffff;
                for (int t = 0; lane + 64 * t < d - 1; ++t) {
                    if ((taken >> t) & 1ull) continue;
                    const float v = sc[lane + 64 * t];
                    if (v > best) { best = v; bi = lane + 64 * t; }
                }
                for (int o = 32; o >= 1; o >>= 1) {
                    const float ob = __shfl_xor(best, o, 64);
                    const int oi = __shfl_xor(bi, o, 64);
                    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
                }
                if (bi != 0x7fffffff && (bi & 63) == lane) taken |= 1ull << (bi >> 6);
                top[u] = bi == 0x7fffffff ? -1 : (bi < p ? bi : bi + 1);   // candidate position
            }
            // Ascending positions, so every S is in lexicographic (id) order.
#pragma unroll
            for (int u = 1; u < kTopMax; ++u)
#pragma unroll
                for (int v = u; v > 0; --v)
                    if (top[v - 1] > top[v] && top[v] >= 0) { const int t = top[v]; top[v] = top[v - 1]; top[v - 1] = t; }
            for (unsigned long long t0 = 0; t0 < nsub; t0 += 64) {
                const unsigned long long t = t0 + lane;
                if (t >= nsub) continue;
                int idx[L];
                comb_unrank<L>(Q, t, idx, SmallBinom());
                int P_[L];
#pragma unroll
                for (int c = 0; c < L; ++c) {
                    int v = -1;
#pragma unroll
                    for (int u = 0; u < kTopMax; ++u) v = idx[c] == u ? top[u] : v;
                    P_[c] = v;
                }
                bool valid = true;
#pragma unroll
                for (int c = 0; c < L; ++c) valid = valid && P_[c] >= 0;
                if (!valid) continue;
                if (!((live_word(adj_row + (j >> 6)) >> (j & 63)) & 1ull)) continue;
                SetFactor<T, L> f;
                f.build(P_, CS, CI);
                int sid[L];
#pragma unroll
                for (int c = 0; c < L; ++c) sid[c] = nb[P_[c]];
                ++my_tests;
                const int dec = f.test(P_, p, CS, CI, tau, tl, band);
                if (dec == 2) {
                    push_recheck<L>(b, pd, row, j, sid, 2);
                } else if (dec == 1) {
                    const int lo = row < j ? row : j, hi = row < j ? j : row;
                    if (take_edge(P.adj, W, lo, hi)) {
                        ++my_removed;
                        write_record(P, lo, hi, L, sid);
                    }
                }
            }
        }
    }
    if (my_tests) add_ll(&s_tests, my_tests);
    if (my_removed) add_ll(&s_removed, my_removed);
    __syncthreads();
    if (tid == 0) {
        Prob &Pw = b.probs[pd];
        if (s_tests) { add_ll(&Pw.tests[L], s_tests); add_ll(&Pw.probe_tests[L], s_tests); }
        if (s_removed) { add_ll(&Pw.removed[L], s_removed); add_ll(&Pw.probe_removed[L], s_removed); }
    }
}

hipError_t launch_feat_plan(hipStream_t s, const Batch &b, long long *foff, long long cap, int *skip) {
    hipLaunchKernelGGL(k_feat_plan, dim3(1), dim3(1024), 0, s, b, foff, cap, skip);
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

template <typename T, int L>
struct ProbeDispatch {
    static hipError_t run(hipStream_t s, const Batch &b, int level, const long long *foff, const float *sc,
                          int topq, const int *skip) {
        if (level == L) {
            hipLaunchKernelGGL((k_probe<T, L>), dim3((unsigned)b.total_rows), dim3(256), 0, s, b, foff, sc, topq,
                               skip);
            return hipGetLastError();
        }
        return ProbeDispatch<T, L + 1>::run(s, b, level, foff, sc, topq, skip);
    }
};
template <typename T>
struct ProbeDispatch<T, kTopMax + 1> {
    static hipError_t run(hipStream_t, const Batch &, int, const long long *, const float *, int, const int *) {
        return hipErrorInvalidValue;
    }
};

hipError_t launch_probe(hipStream_t s, const Batch &b, int level, const long long *foff, const float *scores,
                        int topq, const int *skip) {
    if (level < 1 || level > kTopMax) return hipErrorInvalidValue;
    if (b.prec == PC_PREC_FP64) return ProbeDispatch<double, 1>::run(s, b, level, foff, scores, topq, skip);
    return ProbeDispatch<float, 1>::run(s, b, level, foff, scores, topq, skip);
}

}  // namespace pcg
