/*
 * Oracle for PC-stable skeleton learning with the G^2 test -- TEST
 * INFRASTRUCTURE ONLY (see oracle.h).  Plain C99, single thread, FP64.
 *
 * Parity pins: every function here is checked by the CPU test suite against
 * something other than itself (brute-force counting, high-precision G^2,
 * closed-form and library chi-square tails, itertools order, a d-separation
 * CI oracle on random DAGs, skeleton recovery and label-permutation
 * invariance).  The paper prints no G^2 value, p-value or learned graph, so
 * no pin comes from a printed worked example.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_DEPTHS 256
#define ORC_MAX_CELLS (1LL << 31)

/* ------------------------------------------------------------------------ */
/* Chi-square tail: Q(a, x), the regularised upper incomplete gamma.         */
/*                                                                           */
/* For x < a + 1 the lower function P(a, x) is summed from its power series  */
/*   P(a, x) = x^a e^{-x} / Gamma(a + 1) * sum_{n >= 0} x^n / prod_{k=1..n}(a + k) */
/* and Q = 1 - P.  Otherwise Q is evaluated from Legendre's continued        */
/* fraction for Gamma(a, x),                                                 */
/*   Gamma(a, x) = x^a e^{-x} / (x + 1 - a - 1(1 - a)/(x + 3 - a - 2(2 - a)/(x + 5 - a - ...))) */
/* with the modified Lentz method (Press et al., Numerical Recipes, 6.2).    */
/* ------------------------------------------------------------------------ */

static double lower_series(double a, double x) {
    double term = 1.0 / a; /* x^0 / a, scaled by a so the prefactor uses Gamma(a) */
    double sum = term;
    for (int n = 1; n < 1000000; ++n) {
        term *= x / (a + n);
        sum += term;
        if (fabs(term) < fabs(sum) * DBL_EPSILON) break;
    }
    /* P = x^a e^{-x} / Gamma(a) * sum_{n>=0} x^n / (a (a+1) ... (a+n)) */
    return sum * exp(a * log(x) - x - lgamma(a));
}

static double upper_cfrac(double a, double x) {
    const double tiny = 1e-300;
    /* f = b0 + a1/(b1 + a2/(b2 + ...)), b_k = x + 2k + 1 - a, a_k = -k (k - a) */
    double b = x + 1.0 - a;
    double c = 1.0 / tiny;
    double d = 1.0 / b;
    double f = d;
    for (int k = 1; k < 1000000; ++k) {
        double ak = -(double)k * ((double)k - a);
        b += 2.0;
        d = ak * d + b;
        if (fabs(d) < tiny) d = tiny;
        c = b + ak / c;
        if (fabs(c) < tiny) c = tiny;
        d = 1.0 / d;
        double delta = d * c;
        f *= delta;
        if (fabs(delta - 1.0) < DBL_EPSILON) break;
    }
    /* here f = 1 / (continued fraction); Q = x^a e^{-x} / Gamma(a) * f */
    return f * exp(a * log(x) - x - lgamma(a));
}

double orc_gamma_q(double a, double x) {
    if (!(a > 0.0)) return 1.0;
    if (!(x > 0.0)) return 1.0;
    if (x < a + 1.0) return 1.0 - lower_series(a, x);
    return upper_cfrac(a, x);
}

/* ------------------------------------------------------------------------ */
/* One CI test (Section III-B).                                              */
/* ------------------------------------------------------------------------ */

int orc_ci_test(const uint8_t *data, int64_t m, int32_t n_vars, const uint8_t *cards, int32_t x,
                int32_t y, const int32_t *z, int32_t nz, int64_t *counts_out, double *g2,
                int64_t *df, double *p) {
    return orc_ci_test_ex(data, m, n_vars, cards, x, y, z, nz, ORC_STAT_G2, ORC_DF_DECLARED, counts_out,
                          g2, df, p);
}

int orc_ci_test_ex(const uint8_t *data, int64_t m, int32_t n_vars, const uint8_t *cards, int32_t x,
                   int32_t y, const int32_t *z, int32_t nz, int32_t statistic, int32_t df_rule,
                   int64_t *counts_out, double *stat_out, int64_t *df, double *p) {
    if (statistic != ORC_STAT_G2 && statistic != ORC_STAT_X2) return -1;
    if (df_rule != ORC_DF_DECLARED && df_rule != ORC_DF_ADJUSTED) return -1;
    if (!data || !cards || m < 0 || n_vars <= 0 || nz < 0 || (nz > 0 && !z)) return -1;
    if (x < 0 || x >= n_vars || y < 0 || y >= n_vars || x == y) return -1;
    for (int k = 0; k < nz; ++k)
        if (z[k] < 0 || z[k] >= n_vars || z[k] == x || z[k] == y) return -1;

    const int64_t rx = cards[x], ry = cards[y];
    int64_t nstrata = 1;
    for (int k = 0; k < nz; ++k) {
        nstrata *= cards[z[k]];
        if (nstrata * rx * ry > ORC_MAX_CELLS) return -2;
    }
    const int64_t T = rx * ry * nstrata;
    int64_t *N = (int64_t *)calloc((size_t)(T > 0 ? T : 1), sizeof(int64_t));
    int64_t *Nxz = (int64_t *)calloc((size_t)(rx * nstrata + 1), sizeof(int64_t));
    int64_t *Nyz = (int64_t *)calloc((size_t)(ry * nstrata + 1), sizeof(int64_t));
    int64_t *Nz = (int64_t *)calloc((size_t)(nstrata + 1), sizeof(int64_t));
    if (!N || !Nxz || !Nyz || !Nz) {
        free(N); free(Nxz); free(Nyz); free(Nz);
        return -3;
    }

    /* Contingency table N_xyz: one pass over the samples, one increment each
     * (step (i) of Section IV-A). */
    const uint8_t *cx = data + (int64_t)x * m;
    const uint8_t *cy = data + (int64_t)y * m;
    for (int64_t s = 0; s < m; ++s) {
        int64_t zc = 0, mult = 1;
        for (int k = 0; k < nz; ++k) {
            zc += (int64_t)data[(int64_t)z[k] * m + s] * mult;
            mult *= cards[z[k]];
        }
        N[cx[s] + rx * (cy[s] + ry * zc)] += 1;
    }

    /* Marginals N_x+z, N_+yz, N_++z (step (ii)). */
    for (int64_t zc = 0; zc < nstrata; ++zc)
        for (int64_t yv = 0; yv < ry; ++yv)
            for (int64_t xv = 0; xv < rx; ++xv) {
                int64_t c = N[xv + rx * (yv + ry * zc)];
                Nxz[xv + rx * zc] += c;
                Nyz[yv + ry * zc] += c;
                Nz[zc] += c;
            }

    double G2 = 0.0;
    if (statistic == ORC_STAT_G2) {
        /* G^2 = 2 sum N ln(N / E), E = N_x+z N_+yz / N_++z, over cells with N > 0
         * (0 ln 0 = 0).  Both N * N_++z and N_x+z * N_+yz are formed exactly in
         * int64 (they are below 2^53, so the conversion to double is exact) and
         * the logarithm is taken of their quotient (step (iii)). */
        double sum = 0.0;
        for (int64_t zc = 0; zc < nstrata; ++zc)
            for (int64_t yv = 0; yv < ry; ++yv)
                for (int64_t xv = 0; xv < rx; ++xv) {
                    int64_t c = N[xv + rx * (yv + ry * zc)];
                    if (c == 0) continue;
                    int64_t num = c * Nz[zc];
                    int64_t den = Nxz[xv + rx * zc] * Nyz[yv + ry * zc];
                    sum += (double)c * log((double)num / (double)den);
                }
        G2 = 2.0 * sum;
        if (G2 < 0.0) G2 = 0.0;
    } else {
        /* Pearson's X^2 = sum (N - E)^2 / E over the cells with E > 0, the
         * alternative test of Section II on the same table.  E = 0 only when
         * N_x+z or N_+yz is 0, and then N = 0 too: such cells contribute 0. */
        double sum = 0.0;
        for (int64_t zc = 0; zc < nstrata; ++zc)
            for (int64_t yv = 0; yv < ry; ++yv)
                for (int64_t xv = 0; xv < rx; ++xv) {
                    if (Nz[zc] == 0) continue;
                    double E = (double)Nxz[xv + rx * zc] * (double)Nyz[yv + ry * zc] / (double)Nz[zc];
                    if (E == 0.0) continue;
                    double diff = (double)N[xv + rx * (yv + ry * zc)] - E;
                    sum += diff * diff / E;
                }
        G2 = sum;
    }

    int64_t dof;
    if (df_rule == ORC_DF_DECLARED) {
        /* df = (r_x - 1)(r_y - 1) prod_k r_{z_k}, from the declared cards. */
        dof = (rx - 1) * (ry - 1) * nstrata;
    } else {
        /* Adjusted df: per non-empty stratum, (rows with N_x+z > 0 minus 1)
         * times (columns with N_+yz > 0 minus 1); empty strata add nothing. */
        dof = 0;
        for (int64_t zc = 0; zc < nstrata; ++zc) {
            if (Nz[zc] == 0) continue;
            int64_t a = 0, b = 0;
            for (int64_t xv = 0; xv < rx; ++xv) a += Nxz[xv + rx * zc] > 0;
            for (int64_t yv = 0; yv < ry; ++yv) b += Nyz[yv + ry * zc] > 0;
            dof += (a - 1) * (b - 1);
        }
    }
    double pv = (dof == 0) ? 1.0 : orc_gamma_q(0.5 * (double)dof, 0.5 * G2);

    if (counts_out) memcpy(counts_out, N, (size_t)T * sizeof(int64_t));
    if (stat_out) *stat_out = G2;
    if (df) *df = dof;
    if (p) *p = pv;
    free(N); free(Nxz); free(Nyz); free(Nz);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* PC-stable step 1 (Algorithm 1, with the grouping of Section IV-C).        */
/* ------------------------------------------------------------------------ */

struct orc_result {
    int32_t status;
    int32_t n;
    int32_t n_depths;
    uint8_t *adj;
    int32_t *depth;
    int32_t *sep_off;
    int32_t *pool;
    int64_t pool_len, pool_cap;
    int64_t tests[ORC_MAX_DEPTHS];
    int64_t removed[ORC_MAX_DEPTHS];
    int64_t knife;
    double min_gap;
};

typedef struct {
    const uint8_t *data;
    int64_t m;
    int32_t n;
    const uint8_t *cards;
    int32_t err;
    int32_t statistic, df_rule;
} g2_source;

static double g2_pvalue(void *user, int32_t x, int32_t y, const int32_t *s, int32_t d) {
    g2_source *src = (g2_source *)user;
    double p = 1.0;
    int rc = orc_ci_test_ex(src->data, src->m, src->n, src->cards, x, y, s, d, src->statistic,
                            src->df_rule, NULL, NULL, NULL, &p);
    if (rc != 0 && src->err == 0) src->err = rc;
    return p;
}

static int pool_push(orc_result *r, const int32_t *s, int32_t d) {
    if (r->pool_len + d > r->pool_cap) {
        int64_t cap = r->pool_cap ? 2 * r->pool_cap : 1024;
        while (cap < r->pool_len + d) cap *= 2;
        int32_t *np = (int32_t *)realloc(r->pool, (size_t)cap * sizeof(int32_t));
        if (!np) return -3;
        r->pool = np;
        r->pool_cap = cap;
    }
    memcpy(r->pool + r->pool_len, s, (size_t)d * sizeof(int32_t));
    r->pool_len += d;
    return 0;
}

/* Next size-d subset of positions {0..p-1} in lexicographic order; returns 0
 * when idx already holds the last one. */
static int next_combination(int32_t *idx, int32_t d, int32_t p) {
    int32_t k = d - 1;
    while (k >= 0 && idx[k] == p - d + k) --k;
    if (k < 0) return 0;
    idx[k] += 1;
    for (int32_t l = k + 1; l < d; ++l) idx[l] = idx[l - 1] + 1;
    return 1;
}

/* Runs the tests of one side of an edge: every size-d subset S of cand[0..p)
 * in lexicographic order, stopping at the first p-value above alpha.  Returns
 * 1 when the edge was removed, 0 if not, < 0 on error. */
static int test_side(orc_result *r, int32_t i, int32_t j, const int32_t *cand, int32_t p,
                     int32_t d, double alpha, orc_ci_fn fn, void *user, int32_t *idx,
                     int32_t *S) {
    if (p < d) return 0;
    for (int32_t k = 0; k < d; ++k) idx[k] = k;
    do {
        for (int32_t k = 0; k < d; ++k) S[k] = cand[idx[k]];
        double pv = fn(user, i, j, S, d);
        r->tests[d] += 1;
        double gap = fabs(pv - alpha);
        if (gap < r->min_gap) r->min_gap = gap;
        if (gap < 1e-9) r->knife += 1;
        if (pv > alpha) {
            int32_t n = r->n;
            r->adj[i * n + j] = r->adj[j * n + i] = 0;
            r->depth[i * n + j] = r->depth[j * n + i] = d;
            r->sep_off[i * n + j] = r->sep_off[j * n + i] = (int32_t)r->pool_len;
            if (pool_push(r, S, d) != 0) return -3;
            r->removed[d] += 1;
            return 1;
        }
    } while (d > 0 && next_combination(idx, d, p));
    return 0;
}

orc_result *orc_pc_skeleton_cb(int32_t n, double alpha, int32_t max_depth, orc_ci_fn fn,
                               void *user) {
    orc_result *r = (orc_result *)calloc(1, sizeof(orc_result));
    if (!r) return NULL;
    r->n = n;
    r->min_gap = INFINITY;
    if (n <= 0 || !fn || !(alpha > 0.0 && alpha < 1.0)) {
        r->status = -1;
        return r;
    }
    size_t nn = (size_t)n * (size_t)n;
    r->adj = (uint8_t *)malloc(nn);
    r->depth = (int32_t *)malloc(nn * sizeof(int32_t));
    r->sep_off = (int32_t *)malloc(nn * sizeof(int32_t));
    int32_t *snap = (int32_t *)malloc(nn * sizeof(int32_t)); /* a(v), ascending */
    int32_t *deg = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *candA = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *candB = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *idx = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *S = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!r->adj || !r->depth || !r->sep_off || !snap || !deg || !candA || !candB || !idx || !S) {
        r->status = -3;
        goto done;
    }
    /* Complete undirected graph over the variables. */
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n; ++j) {
            r->adj[i * n + j] = (i != j);
            r->depth[i * n + j] = -1;
            r->sep_off[i * n + j] = -1;
        }

    for (int32_t d = 0; d < ORC_MAX_DEPTHS; ++d) {
        if (max_depth >= 0 && d > max_depth) break;
        /* Freeze a(V) = adj(G, V) for every node before testing (the
         * PC-stable snapshot). */
        for (int32_t v = 0; v < n; ++v) {
            deg[v] = 0;
            for (int32_t u = 0; u < n; ++u)
                if (r->adj[v * n + u]) snap[v * n + deg[v]++] = u;
        }
        /* Stop when no edge has a conditioning set of size d on either side
         * (for d = 0 every surviving pair has its single marginal test). */
        int any = 0;
        for (int32_t i = 0; i < n && !any; ++i)
            for (int32_t j = i + 1; j < n; ++j)
                if (r->adj[i * n + j] && (d == 0 || deg[i] - 1 >= d || deg[j] - 1 >= d)) {
                    any = 1;
                    break;
                }
        if (!any) break;
        r->n_depths = d + 1;

        for (int32_t i = 0; i < n; ++i)
            for (int32_t j = i + 1; j < n; ++j) {
                if (!r->adj[i * n + j]) continue;
                int rc;
                if (d == 0) {
                    /* One marginal test per unordered pair. */
                    rc = test_side(r, i, j, NULL, 0, 0, alpha, fn, user, idx, S);
                } else {
                    int32_t pA = 0, pB = 0;
                    for (int32_t k = 0; k < deg[i]; ++k)
                        if (snap[i * n + k] != j) candA[pA++] = snap[i * n + k];
                    for (int32_t k = 0; k < deg[j]; ++k)
                        if (snap[j * n + k] != i) candB[pB++] = snap[j * n + k];
                    /* The lower-id endpoint's side first; the other side only
                     * if the edge survived it. */
                    rc = test_side(r, i, j, candA, pA, d, alpha, fn, user, idx, S);
                    if (rc == 0) rc = test_side(r, i, j, candB, pB, d, alpha, fn, user, idx, S);
                }
                if (rc < 0) {
                    r->status = rc;
                    goto done;
                }
            }
    }
done:
    free(snap); free(deg); free(candA); free(candB); free(idx); free(S);
    return r;
}

orc_result *orc_pc_skeleton(const uint8_t *data, int64_t m, int32_t n, const uint8_t *cards,
                            double alpha, int32_t max_depth) {
    return orc_pc_skeleton_ex(data, m, n, cards, alpha, max_depth, ORC_STAT_G2, ORC_DF_DECLARED);
}

orc_result *orc_pc_skeleton_ex(const uint8_t *data, int64_t m, int32_t n, const uint8_t *cards,
                               double alpha, int32_t max_depth, int32_t statistic, int32_t df_rule) {
    g2_source src = {data, m, n, cards, 0, statistic, df_rule};
    if (!data || !cards || m <= 0 || n <= 0) {
        orc_result *r = (orc_result *)calloc(1, sizeof(orc_result));
        if (r) r->status = -1;
        return r;
    }
    for (int32_t v = 0; v < n; ++v) {
        if (cards[v] == 0) {
            orc_result *r = (orc_result *)calloc(1, sizeof(orc_result));
            if (r) r->status = -1;
            return r;
        }
    }
    orc_result *r = orc_pc_skeleton_cb(n, alpha, max_depth, g2_pvalue, &src);
    if (r && r->status == 0 && src.err != 0) r->status = src.err;
    return r;
}

int32_t orc_result_status(const orc_result *r) { return r ? r->status : -3; }
int32_t orc_result_n_vars(const orc_result *r) { return r->n; }
int32_t orc_result_n_depths(const orc_result *r) { return r->n_depths; }
int64_t orc_result_tests(const orc_result *r, int32_t d) {
    return (d >= 0 && d < ORC_MAX_DEPTHS) ? r->tests[d] : 0;
}
int64_t orc_result_removed(const orc_result *r, int32_t d) {
    return (d >= 0 && d < ORC_MAX_DEPTHS) ? r->removed[d] : 0;
}
int64_t orc_result_knife_edges(const orc_result *r) { return r->knife; }
double orc_result_min_gap(const orc_result *r) { return r->min_gap; }
void orc_result_export(const orc_result *r, uint8_t *adj, int32_t *depth, int32_t *sep_off) {
    size_t nn = (size_t)r->n * (size_t)r->n;
    if (adj && r->adj) memcpy(adj, r->adj, nn);
    if (depth && r->depth) memcpy(depth, r->depth, nn * sizeof(int32_t));
    if (sep_off && r->sep_off) memcpy(sep_off, r->sep_off, nn * sizeof(int32_t));
}
int64_t orc_result_pool_len(const orc_result *r) { return r->pool_len; }
void orc_result_pool(const orc_result *r, int32_t *pool) {
    if (pool && r->pool_len) memcpy(pool, r->pool, (size_t)r->pool_len * sizeof(int32_t));
}
void orc_result_free(orc_result *r) {
    if (!r) return;
    free(r->adj); free(r->depth); free(r->sep_off); free(r->pool);
    free(r);
}
