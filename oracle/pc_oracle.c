/*
 * Plain FP64 CPU oracle for the skeleton step of order-independent PC (PC-stable).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may include, link or call this file; only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg use it. It shares no code
 * with the HIP library.
 *
 * What it computes, and where the paper defines it (Zarebavani et al., "cuPC: CUDA-based Parallel
 * PC Algorithm for Causal Structure Learning on GPU", IEEE TPDS 2019):
 *   - the skeleton step of PC-stable: level loop, per-level snapshot G' of G, conditioning sets S
 *     drawn from adj(V_i, G') \ {V_j}, removal from G, SepSet storage (Sec. 2.4, Algorithm 1);
 *   - the CI test from the correlation matrix: M0, M1, M2 (Eq. 3), H = M0 - M1 M2^-1 M1^T,
 *     rho = H12 / sqrt(H11 H22) (Eq. 4), Fisher z (Eq. 5) against the threshold of Eq. 6,
 *     "independent" iff z <= tau (Sec. 4.3);
 *   - a Moore-Penrose pseudo-inverse of M2 when it is rank deficient (Sec. 4.4).
 * Readings where the paper is silent or garbled (each is listed with its reason in the project's
 * design notes):
 *   - correlation: Pearson, two-pass mean, C_aa := 1; a constant or non-finite column is an error;
 *   - Phi^-1 by Wichura's algorithm AS241 (PPND16), Applied Statistics 37 (1988) 477-484;
 *   - the level loop runs while (max degree of G) - 1 >= level (the printed "until" is inverted),
 *     capped by max_level; a level with m - level - 3 <= 0 is not run (warning status);
 *   - both directions of an edge are tested: S from adj(i,G')\{j}, then from adj(j,G')\{i};
 *   - canonical order: edges (i<j) lexicographic, direction i first, then subsets of candidate
 *     positions in lexicographic order; the first independent S is stored (ids ascending);
 *   - a tie z == tau removes the edge; |rho| >= 1 is dependent; H11 <= 0 or H22 <= 0 means
 *     rho := 0 (independent);
 *   - M2 is applied through a Cholesky factor; a pivot <= 1e-12 * max diag(M2) switches to the
 *     pseudo-inverse from a symmetric (cyclic Jacobi) eigendecomposition, dropping eigenvalues
 *     <= l * eps64 * lambda_max.
 * The edges of a level may be decided by several threads (oc_set_threads; default one): each
 * decision reads only C and the snapshot G', and the removals and SepSets are applied afterwards
 * in canonical order, so the results do not depend on the thread count.
 */
#include "pc_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------------------------ */
/* Correlation (Pearson, two-pass).                                                           */
/* ------------------------------------------------------------------------------------------ */

/* s_ab / sqrt(s_aa s_bb), the Pearson correlation of two centred columns. The product s_aa s_bb
 * leaves the FP64 range for columns whose scale is beyond about 1e75 (dense SEMs with positive
 * weights reach 1e100), so outside the normal range the two square roots are taken apart. */
static double pearson_ratio(double s_ab, double s_aa, double s_bb)
{
    const double den = s_aa * s_bb;
    if (isfinite(den) && den >= DBL_MIN) return s_ab / sqrt(den);
    return s_ab / (sqrt(s_aa) * sqrt(s_bb));
}

int oc_corr(const double *X, int64_t m, int64_t n, double *C)
{
    if (m < 2 || n < 1) return OC_ERR_SHAPE;
    double *D = (double *)malloc(sizeof(double) * (size_t)m * (size_t)n); /* centred, n x m */
    if (!D) return OC_ERR_ALLOC;
    for (int64_t a = 0; a < n; ++a) {
        double s = 0.0;
        for (int64_t r = 0; r < m; ++r) {
            double x = X[r * n + a];
            if (!isfinite(x)) { free(D); return OC_ERR_NONFINITE; }
            s += x;
        }
        double mu = s / (double)m;
        for (int64_t r = 0; r < m; ++r) D[a * m + r] = X[r * n + a] - mu;
    }
    double *ss = (double *)malloc(sizeof(double) * (size_t)n);
    if (!ss) { free(D); return OC_ERR_ALLOC; }
    for (int64_t a = 0; a < n; ++a) {
        double s = 0.0;
        for (int64_t r = 0; r < m; ++r) s += D[a * m + r] * D[a * m + r];
        if (!(s > 0.0)) { free(D); free(ss); return OC_ERR_CONSTANT; }
        ss[a] = s;
    }
    for (int64_t a = 0; a < n; ++a) {
        C[a * n + a] = 1.0;
        for (int64_t b = a + 1; b < n; ++b) {
            double s = 0.0;
            for (int64_t r = 0; r < m; ++r) s += D[a * m + r] * D[b * m + r];
            const double c = pearson_ratio(s, ss[a], ss[b]);
            C[a * n + b] = c;
            C[b * n + a] = c;
        }
    }
    free(D);
    free(ss);
    return OC_OK;
}

int oc_corr_pair(const double *X, int64_t m, int64_t n, int64_t a, int64_t b, double *out)
{
    if (a == b) { *out = 1.0; return OC_OK; }
    double sa = 0.0, sb = 0.0;
    for (int64_t r = 0; r < m; ++r) { sa += X[r * n + a]; sb += X[r * n + b]; }
    double ma = sa / (double)m, mb = sb / (double)m;
    double saa = 0.0, sbb = 0.0, sab = 0.0;
    for (int64_t r = 0; r < m; ++r) {
        double da = X[r * n + a] - ma, db = X[r * n + b] - mb;
        saa += da * da;
        sbb += db * db;
        sab += da * db;
    }
    if (!(saa > 0.0) || !(sbb > 0.0)) return OC_ERR_CONSTANT;
    *out = pearson_ratio(sab, saa, sbb);
    return OC_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Phi^-1: Wichura's AS241 (PPND16), accurate to about 1e-16 relative.                        */
/* ------------------------------------------------------------------------------------------ */

double oc_ppnd(double p)
{
    if (!(p > 0.0 && p < 1.0)) return NAN;
    double q = p - 0.5;
    if (fabs(q) <= 0.425) {
        double r = 0.180625 - q * q;
        double num = ((((((2.5090809287301226727e+3 * r + 3.3430575583588128105e+4) * r +
                          6.7265770927008700853e+4) * r + 4.5921953931549871457e+4) * r +
                        1.3731693765509461125e+4) * r + 1.9715909503065514427e+3) * r +
                      1.3314166789178437745e+2) * r + 3.3871328727963666080e+0;
        double den = ((((((5.2264952788528545610e+3 * r + 2.8729085735721942674e+4) * r +
                          3.9307895800092710610e+4) * r + 2.1213794301586595867e+4) * r +
                        5.3941960214247511077e+3) * r + 6.8718700749205790830e+2) * r +
                      4.2313330701600911252e+1) * r + 1.0;
        return q * num / den;
    }
    double r = (q < 0.0) ? p : 1.0 - p;
    r = sqrt(-log(r));
    double val;
    if (r <= 5.0) {
        r -= 1.6;
        double num = ((((((7.74545014278341407640e-4 * r + 2.27238449892691845833e-2) * r +
                          2.41780725177450611770e-1) * r + 1.27045825245236838258e+0) * r +
                        3.64784832476320460504e+0) * r + 5.76949722146069140550e+0) * r +
                      4.63033784615654529590e+0) * r + 1.42343711074968357734e+0;
        double den = ((((((1.05075007164441684324e-9 * r + 5.47593808499534494600e-4) * r +
                          1.51986665636164571966e-2) * r + 1.48103976427480074590e-1) * r +
                        6.89767334985100004550e-1) * r + 1.67638483018380384940e+0) * r +
                      2.05319162663775882187e+0) * r + 1.0;
        val = num / den;
    } else {
        r -= 5.0;
        double num = ((((((2.01033439929228813265e-7 * r + 2.71155556874348757815e-5) * r +
                          1.24266094738807843860e-3) * r + 2.65321895265761230930e-2) * r +
                        2.96560571828504891230e-1) * r + 1.78482653991729133580e+0) * r +
                      5.46378491116411436990e+0) * r + 6.65790464350110377720e+0;
        double den = ((((((2.04426310338993978564e-15 * r + 1.42151175831644588870e-7) * r +
                          1.84631831751005468180e-5) * r + 7.86869131145613259100e-4) * r +
                        1.48753612908506148525e-2) * r + 1.36929880922735805310e-1) * r +
                      5.99832206555887937690e-1) * r + 1.0;
        val = num / den;
    }
    return (q < 0.0) ? -val : val;
}

/* Threshold of Eq. 6: tau = Phi^-1(1 - alpha/2) / sqrt(m - |S| - 3). NaN when m - |S| - 3 <= 0. */
double oc_tau(double alpha, double m, int level)
{
    double dof = m - (double)level - 3.0;
    if (!(dof > 0.0)) return NAN;
    return oc_ppnd(1.0 - alpha / 2.0) / sqrt(dof);
}

/* Fisher z of Eq. 5: |0.5 ln((1 + rho) / (1 - rho))|; +inf for |rho| >= 1. */
double oc_fisher_z(double rho)
{
    if (!(fabs(rho) < 1.0)) return INFINITY;
    return fabs(0.5 * log((1.0 + rho) / (1.0 - rho)));
}

/* ------------------------------------------------------------------------------------------ */
/* Symmetric pseudo-inverse (cyclic Jacobi eigendecomposition).                               */
/* ------------------------------------------------------------------------------------------ */

int oc_pinv_sym(const double *A, int k, double *P)
{
    if (k <= 0) return OC_OK;
    double *a = (double *)malloc(sizeof(double) * (size_t)k * (size_t)k);
    double *v = (double *)malloc(sizeof(double) * (size_t)k * (size_t)k);
    if (!a || !v) { free(a); free(v); return OC_ERR_ALLOC; }
    memcpy(a, A, sizeof(double) * (size_t)k * (size_t)k);
    for (int r = 0; r < k; ++r)
        for (int c = 0; c < k; ++c) v[r * k + c] = (r == c) ? 1.0 : 0.0;
    /* Cyclic Jacobi sweeps: rotate away each off-diagonal a[p][q]; stop when it is negligible. */
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int r = 0; r < k; ++r)
            for (int c = 0; c < k; ++c) {
                tot += a[r * k + c] * a[r * k + c];
                if (r != c) off += a[r * k + c] * a[r * k + c];
            }
        if (off <= 1e-32 * tot || off == 0.0) break;
        for (int p = 0; p < k - 1; ++p)
            for (int q = p + 1; q < k; ++q) {
                double apq = a[p * k + q];
                if (apq == 0.0) continue;
                double app = a[p * k + p], aqq = a[q * k + q];
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int r = 0; r < k; ++r) { /* A <- A J (columns p, q) */
                    double arp = a[r * k + p], arq = a[r * k + q];
                    a[r * k + p] = c * arp - s * arq;
                    a[r * k + q] = s * arp + c * arq;
                }
                for (int r = 0; r < k; ++r) { /* A <- J^T A (rows p, q) */
                    double apr = a[p * k + r], aqr = a[q * k + r];
                    a[p * k + r] = c * apr - s * aqr;
                    a[q * k + r] = s * apr + c * aqr;
                }
                for (int r = 0; r < k; ++r) { /* V <- V J */
                    double vrp = v[r * k + p], vrq = v[r * k + q];
                    v[r * k + p] = c * vrp - s * vrq;
                    v[r * k + q] = s * vrp + c * vrq;
                }
            }
    }
    double lmax = 0.0;
    for (int r = 0; r < k; ++r) if (fabs(a[r * k + r]) > lmax) lmax = fabs(a[r * k + r]);
    double cut = (double)k * DBL_EPSILON * lmax;
    for (int r = 0; r < k; ++r)
        for (int c = 0; c < k; ++c) {
            double s = 0.0;
            for (int e = 0; e < k; ++e) {
                double lam = a[e * k + e];
                if (lam > cut) s += v[r * k + e] * v[c * k + e] / lam;
            }
            P[r * k + c] = s;
        }
    free(a);
    free(v);
    return OC_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Partial correlation (Eq. 3-4).                                                             */
/* ------------------------------------------------------------------------------------------ */

int oc_pcor(const double *C, int64_t n, int i, int j, const int *S, int l, double *rho_out)
{
    double h11, h22, h12;
    int used_pinv = 0;
    if (l == 0) {
        h11 = 1.0;
        h22 = 1.0;
        h12 = C[(int64_t)i * n + j];
    } else {
        double *M2 = (double *)malloc(sizeof(double) * (size_t)l * (size_t)l);
        double *L = (double *)calloc((size_t)l * (size_t)l, sizeof(double));
        double *y = (double *)malloc(sizeof(double) * (size_t)l);
        double *w = (double *)malloc(sizeof(double) * (size_t)l);
        if (!M2 || !L || !y || !w) { free(M2); free(L); free(y); free(w); return OC_ERR_ALLOC; }
        for (int a = 0; a < l; ++a)
            for (int b = 0; b < l; ++b) M2[a * l + b] = C[(int64_t)S[a] * n + S[b]];
        double maxdiag = 0.0;
        for (int a = 0; a < l; ++a) if (M2[a * l + a] > maxdiag) maxdiag = M2[a * l + a];
        /* Cholesky M2 = L L^T, row by row. */
        int ok = 1;
        for (int a = 0; a < l && ok; ++a) {
            for (int b = 0; b <= a; ++b) {
                double s = M2[a * l + b];
                for (int e = 0; e < b; ++e) s -= L[a * l + e] * L[b * l + e];
                if (a == b) {
                    if (!(s > 1e-12 * maxdiag)) { ok = 0; break; }
                    L[a * l + a] = sqrt(s);
                } else {
                    L[a * l + b] = s / L[b * l + b];
                }
            }
        }
        if (ok) {
            /* y = L^-1 C(V_i, S)^T, w = L^-1 C(V_j, S)^T; M1 M2^-1 M1^T = [y w]^T [y w]. */
            for (int a = 0; a < l; ++a) {
                double sy = C[(int64_t)i * n + S[a]], sw = C[(int64_t)j * n + S[a]];
                for (int e = 0; e < a; ++e) { sy -= L[a * l + e] * y[e]; sw -= L[a * l + e] * w[e]; }
                y[a] = sy / L[a * l + a];
                w[a] = sw / L[a * l + a];
            }
            double yy = 0.0, ww = 0.0, yw = 0.0;
            for (int a = 0; a < l; ++a) { yy += y[a] * y[a]; ww += w[a] * w[a]; yw += y[a] * w[a]; }
            h11 = 1.0 - yy;
            h22 = 1.0 - ww;
            h12 = C[(int64_t)i * n + j] - yw;
        } else {
            /* Rank-deficient M2: H = M0 - M1 pinv(M2) M1^T. */
            double *P = (double *)malloc(sizeof(double) * (size_t)l * (size_t)l);
            if (!P) { free(M2); free(L); free(y); free(w); return OC_ERR_ALLOC; }
            int st = oc_pinv_sym(M2, l, P);
            if (st != OC_OK) { free(P); free(M2); free(L); free(y); free(w); return st; }
            double q11 = 0.0, q22 = 0.0, q12 = 0.0;
            for (int a = 0; a < l; ++a)
                for (int b = 0; b < l; ++b) {
                    double ci_a = C[(int64_t)i * n + S[a]], cj_a = C[(int64_t)j * n + S[a]];
                    double ci_b = C[(int64_t)i * n + S[b]], cj_b = C[(int64_t)j * n + S[b]];
                    q11 += ci_a * P[a * l + b] * ci_b;
                    q22 += cj_a * P[a * l + b] * cj_b;
                    q12 += ci_a * P[a * l + b] * cj_b;
                }
            h11 = 1.0 - q11;
            h22 = 1.0 - q22;
            h12 = C[(int64_t)i * n + j] - q12;
            used_pinv = 1;
            free(P);
        }
        free(M2);
        free(L);
        free(y);
        free(w);
    }
    if (!(h11 > 0.0) || !(h22 > 0.0)) {
        *rho_out = 0.0;
    } else {
        *rho_out = h12 / sqrt(h11 * h22);
    }
    return used_pinv ? OC_PINV : OC_OK;
}

int oc_ci_test(const double *C, int64_t n, int i, int j, const int *S, int l, double tau,
               double *z_out)
{
    double rho = 0.0;
    int st = oc_pcor(C, n, i, j, S, l, &rho);
    if (st < 0) return st;
    double z = oc_fisher_z(rho);
    if (z_out) *z_out = z;
    return (z <= tau) ? 1 : 0;
}

/* ------------------------------------------------------------------------------------------ */
/* One level of PC-stable (Algorithm 1, one pass of its outer loop).                          */
/* ------------------------------------------------------------------------------------------ */

/* Next combination of l positions out of [0, d) in lexicographic order; returns 0 after the last. */
static int next_combination(int *pos, int l, int d)
{
    int c = l - 1;
    while (c >= 0 && pos[c] == d - l + c) --c;
    if (c < 0) return 0;
    pos[c] += 1;
    for (int e = c + 1; e < l; ++e) pos[e] = pos[e - 1] + 1;
    return 1;
}

/* Tests edge (a, b) from the direction of a: S over adj(a, G') \ {b}. Returns 1 if independent
 * (S written to S_out, ids ascending), 0 if not, negative on error; counts executed tests. */
static int test_direction(const double *C, int64_t n, const unsigned char *Gp, int a, int b, int l,
                          double tau, int *S_out, int64_t *ntests, int *cand, int *pos, int *S)
{
    int d = 0;
    for (int k = 0; k < n; ++k)
        if (k != b && Gp[(int64_t)a * n + k]) cand[d++] = k;
    if (d < l) return 0;
    for (int e = 0; e < l; ++e) pos[e] = e;
    do {
        for (int e = 0; e < l; ++e) S[e] = cand[pos[e]];
        int r = oc_ci_test(C, n, a, b, S, l, tau, NULL);
        *ntests += 1;
        if (r < 0) return r;
        if (r == 1) {
            for (int e = 0; e < l; ++e) S_out[e] = S[e];
            return 1;
        }
    } while (l > 0 && next_combination(pos, l, d));
    return 0;
}

/* Threads of oc_level (1 unless oc_set_threads says otherwise). */
static int g_threads = 1;

void oc_set_threads(int k) { g_threads = k > 0 ? k : 1; }

int oc_level(const double *C, int64_t n, double m, double alpha, int l, unsigned char *G,
             oc_sepset *sep, oc_level_stats *st)
{
    double tau = oc_tau(alpha, m, l);
    if (isnan(tau)) return OC_WARN_SAMPLE_LIMIT;
    unsigned char *Gp = (unsigned char *)malloc((size_t)(n * n));
    if (!Gp) return OC_ERR_ALLOC;
    memcpy(Gp, G, (size_t)(n * n)); /* G' := G */
    /* The edges of G' in canonical order (i < j, lexicographic). */
    int64_t E = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) E += Gp[i * n + j] ? 1 : 0;
    int *ei = (int *)malloc(sizeof(int) * (size_t)(E + 1));
    int *ej = (int *)malloc(sizeof(int) * (size_t)(E + 1));
    int *res = (int *)malloc(sizeof(int) * (size_t)(E + 1));
    int *Sres = (int *)malloc(sizeof(int) * (size_t)(E + 1) * (size_t)(l + 1));
    if (!ei || !ej || !res || !Sres) {
        free(Gp); free(ei); free(ej); free(res); free(Sres);
        return OC_ERR_ALLOC;
    }
    E = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            if (Gp[(int64_t)i * n + j]) { ei[E] = i; ej[E] = j; ++E; }
    /* Every edge is decided from G' alone (Sec. 2.4): S is drawn from the snapshot, and removals
     * go to G only. So the edges may be decided in any order, here by several threads, and the
     * removals and SepSets are then applied in canonical order. */
    int64_t ntests = 0;
    int alloc_fail = 0;
#pragma omp parallel num_threads(g_threads) reduction(+ : ntests)
    {
        int *cand = (int *)malloc(sizeof(int) * (size_t)(n + 1));
        int *pos = (int *)malloc(sizeof(int) * (size_t)(l + 1));
        int *S = (int *)malloc(sizeof(int) * (size_t)(l + 1));
        if (!cand || !pos || !S) {
#pragma omp atomic write
            alloc_fail = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t e = 0; e < E; ++e) {
            if (!cand || !pos || !S) { res[e] = OC_ERR_ALLOC; continue; }
            int *Sbest = Sres + e * (l + 1);
            int r = test_direction(C, n, Gp, ei[e], ej[e], l, tau, Sbest, &ntests, cand, pos, S);
            if (r == 0) r = test_direction(C, n, Gp, ej[e], ei[e], l, tau, Sbest, &ntests, cand, pos, S);
            res[e] = r;
        }
        free(cand); free(pos); free(S);
    }
    int64_t nremoved = 0;
    int status = alloc_fail ? OC_ERR_ALLOC : OC_OK;
    for (int64_t e = 0; e < E && status >= 0; ++e) {
        const int r = res[e];
        if (r < 0) { status = r; break; }
        if (r != 1) continue;
        const int i = ei[e], j = ej[e];
        G[(int64_t)i * n + j] = 0;
        G[(int64_t)j * n + i] = 0;
        nremoved += 1;
        if (sep) {
            if (sep->count < sep->cap) {
                int64_t k = sep->count;
                sep->i[k] = i;
                sep->j[k] = j;
                sep->level[k] = l;
                for (int q = 0; q < l; ++q) sep->S[k * sep->max_level + q] = Sres[e * (l + 1) + q];
            }
            sep->count += 1;
        }
    }
    if (st) {
        st->tests = ntests;
        st->removed = nremoved;
    }
    free(Gp); free(ei); free(ej); free(res); free(Sres);
    return status;
}

int oc_level0(const double *C, int64_t n, double m, double alpha, unsigned char *G,
              oc_level_stats *st)
{
    double tau = oc_tau(alpha, m, 0);
    if (isnan(tau)) return OC_WARN_SAMPLE_LIMIT;
    int64_t removed = 0;
    for (int64_t i = 0; i < n; ++i) {
        G[i * n + i] = 0;
        for (int64_t j = i + 1; j < n; ++j) {
            if (oc_fisher_z(C[i * n + j]) <= tau) {
                G[i * n + j] = 0;
                G[j * n + i] = 0;
                removed += 1;
            } else {
                G[i * n + j] = 1;
                G[j * n + i] = 1;
            }
        }
    }
    if (st) {
        st->tests = n * (n - 1) / 2;
        st->removed = removed;
    }
    return OC_OK;
}

int oc_max_degree(const unsigned char *G, int64_t n)
{
    int best = 0;
    for (int64_t i = 0; i < n; ++i) {
        int d = 0;
        for (int64_t j = 0; j < n; ++j) d += G[i * n + j] ? 1 : 0;
        if (d > best) best = d;
    }
    return best;
}

/* Whole skeleton from a correlation matrix (Algorithm 1). levels_run receives the number of levels
 * executed including level 0; per_level (optional, max_levels entries) receives stats, and
 * G_after (optional, max_levels * n * n bytes) receives G after each level. */
int oc_skeleton_corr(const double *C, int64_t n, double m, double alpha, int max_level,
                     unsigned char *G, oc_sepset *sep, oc_level_stats *per_level, int max_levels,
                     unsigned char *G_after, int *levels_run)
{
    int status = oc_level0(C, n, m, alpha, G, per_level ? &per_level[0] : NULL);
    if (status != OC_OK) return status;
    if (G_after && max_levels > 0) memcpy(G_after, G, (size_t)(n * n));
    int run = 1;
    for (int l = 1;; ++l) {
        if (max_level >= 0 && l > max_level) break;
        if (oc_max_degree(G, n) - 1 < l) break;
        if (!(m - (double)l - 3.0 > 0.0)) { status = OC_WARN_SAMPLE_LIMIT; break; }
        oc_level_stats tmp;
        oc_level_stats *slot = (per_level && l < max_levels) ? &per_level[l] : &tmp;
        status = oc_level(C, n, m, alpha, l, G, sep, slot);
        if (status < 0) return status;
        if (G_after && l < max_levels) memcpy(G_after + (size_t)l * (size_t)(n * n), G, (size_t)(n * n));
        run = l + 1;
    }
    if (levels_run) *levels_run = run;
    return status;
}

int oc_skeleton(const double *X, int64_t m, int64_t n, double alpha, int max_level,
                unsigned char *G, oc_sepset *sep, oc_level_stats *per_level, int max_levels,
                unsigned char *G_after, int *levels_run)
{
    double *C = (double *)malloc(sizeof(double) * (size_t)(n * n));
    if (!C) return OC_ERR_ALLOC;
    int st = oc_corr(X, m, n, C);
    if (st == OC_OK)
        st = oc_skeleton_corr(C, n, (double)m, alpha, max_level, G, sep, per_level, max_levels,
                              G_after, levels_run);
    free(C);
    return st;
}
