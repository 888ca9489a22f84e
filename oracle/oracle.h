/*
 * Oracle for PC-stable skeleton learning with the G^2 test.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded FP64
 * reference written from the paper's definitions.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may call it; the product
 * library never links, loads or calls it, and it shares no code with the GPU
 * path.
 *
 * Sources (Jiang, Wen, Mian, "Fast Parallel Bayesian Network Structure
 * Learning"):
 *   - G^2, expected counts and marginals: Section III-B (the G^2 and E_xyz
 *     definitions).
 *   - df and the p-value decision (p > alpha => independent): Section III-B.
 *   - PC-stable step 1 (snapshot of adjacency sets per depth, edge removal,
 *     SepSet): Section III-C, Algorithm 1.
 *   - Depth 0 has one marginal test per unordered pair: Section IV-B.
 *   - Grouping of the two sides of an edge (adj(V_i)\{V_j} first, then
 *     adj(V_j)\{V_i}, skipped once removed): Section IV-C.
 *   - Lexicographic order of conditioning sets: Section IV-C.
 *
 * Data layout: data[v * n_samples + s], uint8, value in [0, cards[v]).
 */
#ifndef BNS_ORACLE_H
#define BNS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Regularised upper incomplete gamma Q(a, x) = Gamma(a, x) / Gamma(a). */
double orc_gamma_q(double a, double x);

/* One G^2 conditional-independence test I(x, y | z[0..nz)).
 * counts_out (nullable) receives the T = r_x * r_y * prod r_z cells in the
 * layout cell = xv + r_x * (yv + r_y * zc), zc = sum_k zv_k * prod_{l<k} r_{z_l}.
 * Returns 0 on success, -1 on bad arguments, -2 if the table is too large,
 * -3 on allocation failure. */
int orc_ci_test(const uint8_t *data, int64_t n_samples, int32_t n_vars, const uint8_t *cards,
                int32_t x, int32_t y, const int32_t *z, int32_t nz, int64_t *counts_out,
                double *g2, int64_t *df, double *p);

/* Statistic and df rule of orc_ci_test_ex / orc_pc_skeleton_ex. */
enum { ORC_STAT_G2 = 0, ORC_STAT_X2 = 1 };
enum { ORC_DF_DECLARED = 0, ORC_DF_ADJUSTED = 1 };

/* orc_ci_test with a choice of statistic (G^2 of Section III-B, or Pearson's
 * X^2 = sum (N - E)^2 / E over cells with E > 0, named in Section II) and of
 * degrees of freedom (declared: (r_x - 1)(r_y - 1) prod r_z; adjusted: per
 * non-empty stratum z, (#x with N_x+z > 0 - 1)(#y with N_+yz > 0 - 1)).
 * stat_out receives the chosen statistic. */
int orc_ci_test_ex(const uint8_t *data, int64_t n_samples, int32_t n_vars, const uint8_t *cards,
                   int32_t x, int32_t y, const int32_t *z, int32_t nz, int32_t statistic,
                   int32_t df_rule, int64_t *counts_out, double *stat_out, int64_t *df, double *p);

/* A CI decision source for the PC-stable driver: returns a p-value for
 * I(x, y | s[0..d)); the driver declares independence when p > alpha. */
typedef double (*orc_ci_fn)(void *user, int32_t x, int32_t y, const int32_t *s, int32_t d);

typedef struct orc_result orc_result;

/* PC-stable step 1 with the G^2 test on the data.  max_depth < 0: unbounded. */
orc_result *orc_pc_skeleton(const uint8_t *data, int64_t n_samples, int32_t n_vars,
                            const uint8_t *cards, double alpha, int32_t max_depth);

/* Same, with the statistic and df rule of orc_ci_test_ex. */
orc_result *orc_pc_skeleton_ex(const uint8_t *data, int64_t n_samples, int32_t n_vars,
                               const uint8_t *cards, double alpha, int32_t max_depth,
                               int32_t statistic, int32_t df_rule);

/* PC-stable step 1 with an arbitrary CI decision source (used to check the
 * driver against a d-separation oracle). */
orc_result *orc_pc_skeleton_cb(int32_t n_vars, double alpha, int32_t max_depth, orc_ci_fn fn,
                               void *user);

int32_t orc_result_status(const orc_result *r);    /* 0 ok, <0 as orc_ci_test */
int32_t orc_result_n_vars(const orc_result *r);
int32_t orc_result_n_depths(const orc_result *r);  /* depths at which tests ran */
int64_t orc_result_tests(const orc_result *r, int32_t d);    /* tests run at depth d */
int64_t orc_result_removed(const orc_result *r, int32_t d);  /* edges removed at depth d */
int64_t orc_result_knife_edges(const orc_result *r);  /* tests with |p - alpha| < 1e-9 */
double orc_result_min_gap(const orc_result *r);       /* min |p - alpha| over all tests */
/* adj: n*n uint8 (final skeleton).  depth: n*n int32 (removal depth, -1 kept).
 * sep_off: n*n int32 offset of the sepset in pool (-1 none); sepset of a pair
 * removed at depth d is pool[off .. off + d), ascending variable ids. */
void orc_result_export(const orc_result *r, uint8_t *adj, int32_t *depth, int32_t *sep_off);
int64_t orc_result_pool_len(const orc_result *r);
void orc_result_pool(const orc_result *r, int32_t *pool);
void orc_result_free(orc_result *r);

#ifdef __cplusplus
}
#endif
#endif
