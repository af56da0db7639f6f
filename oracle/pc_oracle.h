/*
 * Plain FP64 CPU oracle for the PC-stable skeleton. TEST INFRASTRUCTURE ONLY: used by the test
 * suite, the smoke check and the benchmark's CPU-baseline leg, never by the product path.
 */
#ifndef PC_ORACLE_H
#define PC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    OC_OK = 0,
    OC_PINV = 1,               /* oc_pcor: result used the pseudo-inverse path */
    OC_WARN_SAMPLE_LIMIT = 2,  /* a level was not run because m - level - 3 <= 0 */
    OC_ERR_SHAPE = -1,
    OC_ERR_CONSTANT = -2,
    OC_ERR_NONFINITE = -3,
    OC_ERR_ALLOC = -4,
};

/* SepSet records: record k is (i[k] < j[k], level[k], S[k*max_level .. +level) ids ascending).
 * count may exceed cap; records past cap are counted but not stored. Level-0 SepSets (empty) are
 * not recorded. */
typedef struct {
    int32_t *i, *j, *level, *S;
    int64_t cap, count;
    int32_t max_level;
} oc_sepset;

typedef struct {
    int64_t tests;    /* CI tests executed in canonical order with early stop per edge */
    int64_t removed;  /* edges removed in this level */
} oc_level_stats;

int oc_corr(const double *X, int64_t m, int64_t n, double *C);
int oc_corr_pair(const double *X, int64_t m, int64_t n, int64_t a, int64_t b, double *out);
double oc_ppnd(double p);
double oc_tau(double alpha, double m, int level);
double oc_fisher_z(double rho);
int oc_pinv_sym(const double *A, int k, double *P);
int oc_pcor(const double *C, int64_t n, int i, int j, const int *S, int l, double *rho_out);
int oc_ci_test(const double *C, int64_t n, int i, int j, const int *S, int l, double tau,
               double *z_out);
/* Threads oc_level uses (default 1); results do not depend on it. */
void oc_set_threads(int k);
int oc_level0(const double *C, int64_t n, double m, double alpha, unsigned char *G,
              oc_level_stats *st);
int oc_level(const double *C, int64_t n, double m, double alpha, int l, unsigned char *G,
             oc_sepset *sep, oc_level_stats *st);
int oc_max_degree(const unsigned char *G, int64_t n);
int oc_skeleton_corr(const double *C, int64_t n, double m, double alpha, int max_level,
                     unsigned char *G, oc_sepset *sep, oc_level_stats *per_level, int max_levels,
                     unsigned char *G_after, int *levels_run);
int oc_skeleton(const double *X, int64_t m, int64_t n, double alpha, int max_level,
                unsigned char *G, oc_sepset *sep, oc_level_stats *per_level, int max_levels,
                unsigned char *G_after, int *levels_run);

#ifdef __cplusplus
}
#endif
#endif
