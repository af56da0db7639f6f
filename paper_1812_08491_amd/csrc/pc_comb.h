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
template <int L, typename Binom>
__host__ __device__ inline void comb_unrank(int d, unsigned long long t, int (&P)[L > 0 ? L : 1],
                                            const Binom &binom) {
    int x = 0;
#pragma unroll
    for (int c = 0; c < L; ++c) {
        for (; x < d; ++x) {  // x < d always holds for t < C(d, L); the bound is a guard
            unsigned long long cnt = binom(d - 1 - x, L - 1 - c);
            if (t < cnt) break;
            t -= cnt;
        }
        P[c] = x;
        ++x;
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
