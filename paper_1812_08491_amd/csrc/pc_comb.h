// Combination function of Sec. 4.2 (Algorithm 6, "ParComb", after Buckles and Lybanon): the t-th
// l-subset of {0, .., d-1} in lexicographic order, computed directly from t.
//
// Eq. 7 writes t as the sum, over the subset's elements in order, of the number of subsets that
// start with a smaller element at that position: skipping value v at position c passes over
// C(d-1-v, l-1-c) subsets. Walking v upward while that count does not exceed what is left of t
// yields the elements one by one (the paper's 1-based values minus one, as it prescribes).
//
// Shared by the device code and by the host helper pc_comb_unrank (which the CPU tests pin against
// the paper's printed examples), so the same function is checked and used.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcg {

// binom(a, b) must return C(a, b), and 0 when a < b. L is the subset size; t < C(d, L).
//
// Same function as the walk described above, with fewer table reads: the subsets whose element at
// position c is below y, given elements before it and smallest candidate x, number
// C(d - x, k) - C(d - y, k) with k = L - c (the hockey-stick identity summed over the skipped
// values), so the element is the largest y with that count <= t, found by bisection when the
// candidate range is long and by the step-by-step walk when it is short. At L = 1 the element is t.
template <int L, typename Binom>
__host__ __device__ inline void comb_unrank(int d, unsigned long long t, int (&P)[L > 0 ? L : 1],
                                            const Binom &binom) {
    if constexpr (L == 1) {
        P[0] = (int)t;
        return;
    }
    int x = 0;
#pragma unroll
    for (int c = 0; c < L; ++c) {
        const int k = L - c;
        int lo = x, hi = d - k;   // the element lies in [lo, hi] for t < C(d - x, k)
        if (hi - lo >= 8) {
            const unsigned long long top = binom(d - x, k);
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (top - binom(d - mid, k) <= t) lo = mid;
                else hi = mid - 1;
            }
            t -= top - binom(d - lo, k);
        } else {
            for (; lo < hi; ++lo) {
                const unsigned long long cnt = binom(d - 1 - lo, k - 1);
                if (t < cnt) break;
                t -= cnt;
            }
        }
        P[c] = lo;
        x = lo + 1;
    }
}

// Lexicographic successor of P (ascending positions below d); returns false after the last subset.
template <int L>
__host__ __device__ inline bool comb_next(int d, int (&P)[L > 0 ? L : 1]) {
    int pos = -1;
#pragma unroll
    for (int c = L - 1; c >= 0; --c)
        if (pos < 0 && P[c] < d - L + c) pos = c;
    if (pos < 0) return false;
#pragma unroll
    for (int c = 0; c < L; ++c) {
        if (c == pos) P[c] += 1;
        else if (c > pos) P[c] = P[c - 1] + 1;
    }
    return true;
}

}  // namespace pcg
