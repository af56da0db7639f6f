// The CI test of Eq. 3-6 for one conditioning set S shared across the j of a row (the sharing of
// cuPC-S, Sec. 3.4), plus the edge-removal and queue helpers used by the level and probe kernels.
#pragma once

#include "pc_dev.h"

namespace pcg {

__device__ inline double fisher_z64(double r) {
    if (!(fabs(r) < 1.0)) return INFINITY;
    return fabs(0.5 * log((1.0 + r) / (1.0 - r)));
}

__device__ inline unsigned long long live_word(unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// Writes one SepSet record: (lo, hi, level) and S[0..level), the rest -1.
__device__ inline void store_record(pc_sep_rec *rec, int lo, int hi, int level, const int *S) {
    rec->i = lo;
    rec->j = hi;
    rec->level = level;
    for (int c = 0; c < PC_MAX_LEVEL; ++c) rec->S[c] = c < level ? S[c] : -1;
}

// Appends the SepSet record of the removed edge (lo, hi). The lanes of a wavefront that reach this
// call together take consecutive slots with a single atomic add by the lowest of them, which keeps
// the shared counter from serialising one device-scope atomic per removal. All active lanes must
// be working on the same problem P.
__device__ inline void write_record(const Prob &P, int lo, int hi, int level, const int *S) {
    const unsigned long long act = __ballot(1);
    const int lane = (int)__lane_id();
    const int leader = __ffsll((long long)act) - 1;
    unsigned long long base = 0ull;
    if (lane == leader)
        base = atomicAdd(reinterpret_cast<unsigned long long *>(P.rec_count), (unsigned long long)__popcll(act));
    base = __shfl(base, leader, 64);
    const long long k = (long long)(base + (unsigned long long)__popcll(act & ((1ull << lane) - 1ull)));
    if (k < P.rec_cap) store_record(P.recs + k, lo, hi, level, S);
}

// Pushes a test to the re-check queue; cls is the FP32 classification (0 dependent, 1 independent,
// 2 inside the band). The lanes of a wavefront that reach this call together reserve consecutive
// slots with one atomic add by the lowest of them, in the queue slice of their work-group: same-
// address device atomics serialise, and a level can push millions of tests (BF16x3 bands). Lanes
// that find the slice full move on to the next slices; only when every slice is full is the test
// dropped and the overflow flagged.
template <int L>
__device__ inline void push_recheck(const Batch &b, int d, int row, int j, const int (&sid)[L], int cls) {
    // Once the queue has overflowed, the level will be redone: further pushes are moot.
    if (__hip_atomic_load(&b.st->rq_overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int lane = (int)__lane_id();
    const unsigned long long cap_s = (unsigned long long)(b.rq_cap / kRqSlices);
    unsigned long long act = __ballot(1);          // lanes still without a slot (uniform)
    int slice = (int)(blockIdx.x % kRqSlices);
    long long pos = -1;
    for (int tries = 0; tries < kRqSlices && act; ++tries) {
        const int leader = __ffsll((long long)act) - 1;
        unsigned long long base = 0ull;
        if (lane == leader) base = atomicAdd(&b.st->rq_slice[slice], (unsigned long long)__popcll(act));
        base = __shfl(base, leader, 64);
        if (pos < 0 && ((act >> lane) & 1ull)) {
            const unsigned long long k = base + (unsigned long long)__popcll(act & ((1ull << lane) - 1ull));
            if (k < cap_s) pos = (long long)((unsigned long long)slice * cap_s + k);
        }
        act = __ballot(pos < 0);
        slice = slice + 1 == kRqSlices ? 0 : slice + 1;
    }
    if (pos < 0) {
        // The level's result would be incomplete: record it and stop the level loop, so that the
        // host can redo this level (in FP64) from its snapshot G', which no later level overwrote.
        atomicMax(&b.st->rq_overflow, L);
        b.st->done = 1;
        return;
    }
    RqEntry *e = b.rq + pos;
    e->prob = d;
    e->i = row;
    e->j = j;
    e->cls = cls;
#pragma unroll
    for (int c = 0; c < PC_MAX_LEVEL; ++c) e->S[c] = c < L ? (uint16_t)sid[c] : (uint16_t)0xffff;
}

// Factor of M2 = C[S,S] for one S (positions P into the row's neighbour list), shared by all j.
template <typename T, int L>
struct SetFactor {
    T Lm[L * (L + 1) / 2];
    T rd[L];
    T y[L];
    T h11;
    float g2;   // (1 + sqrt(l tr(M2^-1)))^2: amplification of C errors into rho (FP32 band)
    bool ok;    // all Cholesky pivots above the tolerance

    // cs(p, q) = C[N_p, N_q] (1 on the diagonal), ci(p) = C[i, N_p].
    template <class CS, class CI>
    __device__ inline void build(const int (&P)[L], const CS &cs, const CI &ci) {
        ok = true;
#pragma unroll
        for (int r = 0; r < L; ++r) {
#pragma unroll
            for (int c = 0; c <= r; ++c) {
                T s = cs(P[r], P[c]);
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
            T s = ci(P[r]);
#pragma unroll
            for (int e = 0; e < r; ++e) s -= Lm[r * (r + 1) / 2 + e] * y[e];
            y[r] = s * rd[r];
            yy += y[r] * y[r];
        }
        h11 = (T)1 - yy;
        g2 = 4.0f;
        if (sizeof(T) == 4 && L > 1) {
            // g = 1 + sqrt(l tr(M2^-1)) bounds 1 + ||M2^-1 c||_1 for any c with c^T M2^-1 c <= 1,
            // where tr(M2^-1) = ||L^-1||_F^2.
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
    }

    // Test of edge (i, N_p) given S: 0 dependent, 1 independent, 2 to be re-checked in FP64
    // (inside the FP32 error band, or M2 rank deficient).
    template <class CS, class CI>
    __device__ inline int test(const int (&P)[L], int p, const CS &cs, const CI &ci, double tau,
                               float tl, float band) const {
        T col[L];
#pragma unroll
        for (int r = 0; r < L; ++r) col[r] = cs(p, P[r]);
        return test_vals(col, ci(p), tau, tl, band);
    }

    // The same test from values already loaded: col[r] = C[N_p, S_r], cij = C[i, N_p].
    __device__ inline int test_vals(const T (&col)[L], T cij, double tau, float tl, float band) const {
        T w[L];
        T ww = 0, yw = 0;
#pragma unroll
        for (int r = 0; r < L; ++r) {
            T s = col[r];
#pragma unroll
            for (int e = 0; e < r; ++e) s -= Lm[r * (r + 1) / 2 + e] * w[e];
            w[r] = s * rd[r];
            ww += w[r] * w[r];
            yw += y[r] * w[r];
        }
        const T h22 = (T)1 - ww;
        const T h12 = cij - yw;
        if (sizeof(T) == 8) {
            if (!ok) return 2;  // rank-deficient M2: pseudo-inverse path of the re-check kernel
            const double rho = (h11 > 0 && h22 > 0) ? (double)h12 / sqrt((double)h11 * (double)h22) : 0.0;
            return fisher_z64(rho) <= tau ? 1 : 0;
        }
        // Errors dC in the entries of C move H12 by up to dC (1 + |M2^-1 c_iS|_1)(1 + |M2^-1 c_jS|_1)
        // and H11, H22 by the squares. At l = 1 (M2 = [1]) these factors are 1 + |C_ik| and
        // 1 + |C_jk| exactly; above, g bounds both.
        float gi2 = g2, gj2 = g2, gij = g2;
        if (L == 1) {
            const float gi = 1.0f + fabsf((float)y[0]), gj = 1.0f + fabsf((float)w[0]);
            gi2 = gi * gi;
            gj2 = gj * gj;
            gij = gi * gj;
        }
        const float fh11 = (float)h11, fh22 = (float)h22;
        if (!ok || fh11 <= 2.0f * band * gi2 || fh22 <= 2.0f * band * gj2) return 2;
        // v_rsq_f32 and v_rcp_f32 (1 ulp each): both pivots exceed 2 band > 0 here, far from the
        // denormal range, so no input scaling is needed. err bounds the FP32 error of ar; it is
        // inflated by 2^-16 so that the rounding of its own few operations cannot leave it short.
        const float inv = __builtin_amdgcn_rsqf(fh11 * fh22);
        const float ar = fabsf((float)h12 * inv);
        const float err = band * (gij * inv + 0.5f * ar * (gi2 * __builtin_amdgcn_rcpf(fh11) +
                                                            gj2 * __builtin_amdgcn_rcpf(fh22))) *
                          (1.0f + 0x1p-16f);
        return ar <= tl - err ? 1 : (ar > tl + err ? 0 : 2);
    }
};

}  // namespace pcg
