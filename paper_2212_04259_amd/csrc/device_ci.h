// Device-side building blocks of one G^2 conditional-independence test on
// gfx950: LDS-histogram counting of the contingency table, marginals, the
// G^2 log-sum, the FP64 chi-square tail and the FP64 re-check.
//
// Definitions followed (Jiang, Wen, Mian, Section III-B): N_xyz counts the
// samples with X = x, Y = y, Z = z; E_xyz = N_x+z N_+yz / N_++z;
// G^2 = 2 sum N ln(N / E); p from the chi-square distribution with
// (r_X - 1)(r_Y - 1) prod r_Z degrees of freedom; independence iff p > alpha.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bns_internal.h"

namespace bns {

// ---------------------------------------------------------------------------
// Per-test description staged in LDS (filled by the kernel before a test).
// ---------------------------------------------------------------------------
struct TestSh {
    const uint8_t *col[kMaxCols];  // x, y, z_1..z_d columns
    uint32_t card[kMaxCols];
    uint32_t mult[kMaxCols];       // cell stride of each column: 1, r_x, r_x r_y, ...
    int32_t ncols;                 // d + 2
    int32_t pad;
    int64_t m;                     // samples
    double red_d[kWaves];
    float red_f[kWaves];
    double bcast_d[2];
    int32_t bcast_i[4];
};

struct TestOut {
    double g2;
    double p;
    int64_t df;
    int32_t flags;   // bit 0 independent, bit 1 rechecked
    int32_t err;     // DevError
};

// ---------------------------------------------------------------------------
// Workgroup reductions in a fixed order (deterministic results).
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double wg_sum(double v, TestSh &t) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) t.red_d[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += t.red_d[w];
    __syncthreads();
    return s;
}

__device__ inline float wg_sum(float v, TestSh &t) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) t.red_f[threadIdx.x >> 6] = v;
    __syncthreads();
    float s = 0.0f;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += t.red_f[w];
    __syncthreads();
    return s;
}

// Exact quotient i / d for i < 2^24 via a float reciprocal and one correction.
__device__ inline uint32_t fast_div(uint32_t i, uint32_t d, float inv) {
    uint32_t q = (uint32_t)((float)i * inv);
    if (q * d > i) {
        --q;
    } else if ((q + 1) * d <= i) {
        ++q;
    }
    return q;
}

// ---------------------------------------------------------------------------
// Chi-square upper tail in FP64: p = Q(a, x) with a = df/2, x = G^2/2.
// Lower regularised gamma from its power series when x < a + 1, else the
// upper one from the Legendre continued fraction (modified Lentz).
// ---------------------------------------------------------------------------
static __device__ __noinline__ double chi2_upper(int64_t df, double g2) {
    if (df <= 0) return 1.0;
    const double a = 0.5 * (double)df;
    const double x = 0.5 * g2;
    if (!(x > 0.0)) return 1.0;
    const double log_front = a * log(x) - x - lgamma(a);  // log(x^a e^-x / Gamma(a))
    if (x < a + 1.0) {
        // gamma(a,x)/Gamma(a) = x^a e^-x / Gamma(a) * sum_k x^k / (a (a+1) ... (a+k))
        double term = 1.0 / a, acc = term, den = a;
        for (int k = 0; k < 200000; ++k) {
            den += 1.0;
            term *= x / den;
            acc += term;
            if (term <= acc * 1.1102230246251565e-16) break;
        }
        double lower = exp(log_front) * acc;
        return lower >= 1.0 ? 0.0 : 1.0 - lower;
    }
    // Gamma(a,x)/Gamma(a) = x^a e^-x / Gamma(a) / (x+1-a - 1(1-a)/(x+3-a - 2(2-a)/(x+5-a - ...)))
    const double fpmin = 1e-300;
    double bk = x + 1.0 - a;
    double C = 1.0 / fpmin;
    double D = 1.0 / bk;
    double H = D;
    for (int k = 1; k < 200000; ++k) {
        const double ak = (double)k * (a - (double)k);
        bk += 2.0;
        D = bk + ak * D;
        D = (fabs(D) < fpmin) ? fpmin : D;
        C = bk + ak / C;
        C = (fabs(C) < fpmin) ? fpmin : C;
        D = 1.0 / D;
        const double step = C * D;
        H *= step;
        if (fabs(step - 1.0) <= 2.220446049250313e-16) break;
    }
    return exp(log_front) * H;
}

// Density of Gamma(a, 1) at x (the derivative of Q(a, x) in x, up to sign).
static __device__ __noinline__ double gamma_density(double a, double x) {
    if (!(x > 0.0)) return 0.0;
    return exp((a - 1.0) * log(x) - x - lgamma(a));
}

// ---------------------------------------------------------------------------
// One cell's share of G^2 / 2 in a form whose terms are all non-negative.
//
// Within a stratum z with N_++z > 0, sum_{x,y} (N_xyz - E_xyz) = 0, so
//   G^2 / 2 = sum_{N>0} N ln(N/E) = sum_{N>0} [N ln(N/E) - N + E] + sum_{N=0} E
//           = sum_{N>0} N (w - 1 - ln w) + sum_{N=0} E,   w = E / N.
// Each summand is >= 0, so a low-precision sum has no cancellation.  With
// a = N N_++z and b = N_x+z N_+yz (exact integers), w = b / a and
// t = (a - b) / (a + b) gives w - 1 - ln w = 2t^2/(1+t) + 2 sum_k t^(2k+1)/(2k+1),
// k >= 1, used when |t| is small; the direct form is used otherwise.
// ---------------------------------------------------------------------------
template <typename Real>
struct TermCfg;
template <>
struct TermCfg<float> {
    static constexpr float tau = 0.3334f;
    static constexpr int terms = 7;
};
template <>
struct TermCfg<double> {
    static constexpr double tau = 0.1;
    static constexpr int terms = 8;
};

template <typename Real>
__device__ inline Real g2_half_term(uint32_t N, uint32_t nxz, uint32_t nyz, uint32_t nzz) {
    if (N == 0) return (Real)nxz * (Real)nyz / (Real)nzz;
    const uint64_t a = (uint64_t)N * nzz;
    const uint64_t b = (uint64_t)nxz * nyz;
    const Real t = (Real)((int64_t)a - (int64_t)b) / (Real)(a + b);
    if (fabs(t) <= TermCfg<Real>::tau) {
        const Real u = t * t;
        Real s = (Real)1 / (Real)(2 * TermCfg<Real>::terms + 1);
#pragma unroll
        for (int k = TermCfg<Real>::terms - 1; k >= 1; --k) s = s * u + (Real)1 / (Real)(2 * k + 1);
        // s = sum_{k>=1} t^(2k-2) / (2k+1)
        return (Real)N * ((Real)2 * u / ((Real)1 + t) + (Real)2 * t * u * s);
    }
    const Real w = (Real)b / (Real)a;
    return (Real)N * (w - (Real)1 - log(w));
}

// ---------------------------------------------------------------------------
// Counting (step (i) of Section IV-A) into an LDS table.
//
// Columns are uint8, read 16 samples per lane per column with coalesced
// 16-byte loads.  Cell of a sample: sum_k value_k * mult_k.  Only cells in
// [cbase, cbase + Tc) are counted (z-range chunking of large tables).  The
// table is replicated 2^logR times, interleaved per cell (replica = lane bits)
// so that lanes hitting the same cell usually hit different LDS words.
// ---------------------------------------------------------------------------
__device__ inline uint32_t byte_of(const uint4 &v, int b) {
    const uint32_t w = (b < 4) ? v.x : (b < 8) ? v.y : (b < 12) ? v.z : v.w;
    return (w >> (8 * (b & 3))) & 0xffu;
}

template <int NC>
__device__ inline void count_fixed(const TestSh &t, uint32_t *tab, uint32_t cbase, uint32_t Tc,
                                   int logR, int64_t q0, int64_t q1) {
    const uint32_t rep = threadIdx.x & ((1u << logR) - 1u);
    const uint4 *cp[NC];
    uint32_t mul[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        cp[k] = reinterpret_cast<const uint4 *>(t.col[k]);
        mul[k] = t.mult[k];
    }
    for (int64_t q = q0 + threadIdx.x; q < q1; q += kWG) {
        uint4 v[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) v[k] = cp[k][q];
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            uint32_t cell = byte_of(v[0], b);
#pragma unroll
            for (int k = 1; k < NC; ++k) cell += __umul24(byte_of(v[k], b), mul[k]);
            const uint32_t idx = cell - cbase;
            if (idx < Tc) atomicAdd(&tab[(idx << logR) | rep], 1u);
        }
    }
}

__device__ inline void count_generic(const TestSh &t, uint32_t *tab, uint32_t cbase, uint32_t Tc,
                                     int logR, int64_t q0, int64_t q1) {
    const uint32_t rep = threadIdx.x & ((1u << logR) - 1u);
    const int nc = t.ncols;
    for (int64_t q = q0 + threadIdx.x; q < q1; q += kWG) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            uint32_t cell[4];
            {
                const uint32_t v = reinterpret_cast<const uint32_t *>(t.col[0])[4 * q + w];
#pragma unroll
                for (int b = 0; b < 4; ++b) cell[b] = (v >> (8 * b)) & 0xffu;
            }
            for (int k = 1; k < nc; ++k) {
                const uint32_t v = reinterpret_cast<const uint32_t *>(t.col[k])[4 * q + w];
                const uint32_t mk = t.mult[k];
#pragma unroll
                for (int b = 0; b < 4; ++b) cell[b] += __umul24((v >> (8 * b)) & 0xffu, mk);
            }
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const uint32_t idx = cell[b] - cbase;
                if (idx < Tc) atomicAdd(&tab[(idx << logR) | rep], 1u);
            }
        }
    }
}

// Samples [s0, s1) one byte at a time (the ragged tail after the 16-sample groups).
__device__ inline void count_tail(const TestSh &t, uint32_t *tab, uint32_t cbase, uint32_t Tc,
                                  int logR, int64_t s0, int64_t s1) {
    const uint32_t rep = threadIdx.x & ((1u << logR) - 1u);
    for (int64_t s = s0 + threadIdx.x; s < s1; s += kWG) {
        uint32_t cell = t.col[0][s];
        for (int k = 1; k < t.ncols; ++k) cell += __umul24((uint32_t)t.col[k][s], t.mult[k]);
        const uint32_t idx = cell - cbase;
        if (idx < Tc) atomicAdd(&tab[(idx << logR) | rep], 1u);
    }
}

// Counts samples [s0, s1) (s0 a multiple of 16).
__device__ inline void count_samples(const TestSh &t, uint32_t *tab, uint32_t cbase, uint32_t Tc,
                                     int logR, int64_t s0, int64_t s1) {
    const int64_t q0 = s0 >> 4, q1 = s1 >> 4;
    switch (t.ncols) {
        case 2: count_fixed<2>(t, tab, cbase, Tc, logR, q0, q1); break;
        case 3: count_fixed<3>(t, tab, cbase, Tc, logR, q0, q1); break;
        case 4: count_fixed<4>(t, tab, cbase, Tc, logR, q0, q1); break;
        case 5: count_fixed<5>(t, tab, cbase, Tc, logR, q0, q1); break;
        case 6: count_fixed<6>(t, tab, cbase, Tc, logR, q0, q1); break;
        default: count_generic(t, tab, cbase, Tc, logR, q0, q1); break;
    }
    if ((q1 << 4) < s1) count_tail(t, tab, cbase, Tc, logR, q1 << 4, s1);
}

// Sums the 2^logR interleaved replicas of each cell: out[c] = sum_r rep[c * R + r].
__device__ inline void reduce_replicas(const uint32_t *rep_tab, uint32_t *out, uint32_t Tc,
                                       int logR) {
    const uint32_t R = 1u << logR;
    const uint32_t total = Tc << logR;
    const uint32_t lane = threadIdx.x & 63u;
    for (uint32_t base = (threadIdx.x & ~63u); base < total; base += kWG) {
        const uint32_t e = base + lane;
        uint32_t v = (e < total) ? rep_tab[e] : 0u;
        for (uint32_t off = 1; off < R; off <<= 1) v += __shfl_xor(v, (int)off, 64);
        if ((lane & (R - 1u)) == 0u && e < total) out[e >> logR] = v;
    }
}

// Marginal tables of a chunk of Zc strata (step (ii) of Section IV-A):
// rows[x + rx z] = N_x+z, cols[y + ry z] = N_+yz, strata[z] = N_++z.
__device__ inline void marginals(const uint32_t *tab, uint32_t *rows, uint32_t *cols,
                                 uint32_t *strata, uint32_t rx, uint32_t ry, uint32_t Zc) {
    const float inv_rx = 1.0f / (float)rx;
    const uint32_t nrow = rx * Zc, ncol = ry * Zc;
    for (uint32_t i = threadIdx.x; i < nrow + ncol; i += kWG) {
        if (i < nrow) {
            const uint32_t z = fast_div(i, rx, inv_rx), xv = i - z * rx;
            const uint32_t *p = tab + xv + rx * ry * z;
            uint32_t s = 0;
            for (uint32_t yv = 0; yv < ry; ++yv) s += p[rx * yv];
            rows[i] = s;
        } else {
            const uint32_t rho = i - nrow;
            const uint32_t *p = tab + rx * rho;
            uint32_t s = 0;
            for (uint32_t xv = 0; xv < rx; ++xv) s += p[xv];
            cols[rho] = s;
        }
    }
    __syncthreads();
    for (uint32_t z = threadIdx.x; z < Zc; z += kWG) {
        uint32_t s = 0;
        for (uint32_t yv = 0; yv < ry; ++yv) s += cols[yv + ry * z];
        strata[z] = s;
    }
    __syncthreads();
}

// This thread's part of sum of g2_half_term over the chunk.
template <typename Real>
__device__ inline Real g2_partial(const uint32_t *tab, const uint32_t *rows, const uint32_t *cols,
                                  const uint32_t *strata, uint32_t rx, uint32_t ry, uint32_t Zc) {
    const float inv_ry = 1.0f / (float)ry;
    Real acc = 0;
    for (uint32_t rho = threadIdx.x; rho < ry * Zc; rho += kWG) {
        const uint32_t z = fast_div(rho, ry, inv_ry);
        const uint32_t nzz = strata[z];
        if (nzz == 0) continue;
        const uint32_t nyz = cols[rho];
        const uint32_t *trow = tab + rx * rho;
        const uint32_t *mrow = rows + rx * z;
        for (uint32_t xv = 0; xv < rx; ++xv) acc += g2_half_term<Real>(trow[xv], mrow[xv], nyz, nzz);
    }
    return acc;
}

// ---------------------------------------------------------------------------
// Chunk plan of a test: how many strata fit per LDS pass and the replication.
// ---------------------------------------------------------------------------
struct Plan {
    uint32_t rx, ry, rxy;
    uint32_t nstrata;     // prod r_z
    uint32_t T;           // cells
    uint32_t zc_per;      // strata per chunk
    uint32_t nchunks;
    int logR;             // replication of single-chunk tables
    int64_t df;
    int32_t err;
};

__device__ inline Plan make_plan(const TestSh &t, const Tile &tile) {
    Plan P;
    P.err = kDevOk;
    P.rx = t.card[0];
    P.ry = t.card[1];
    P.rxy = P.rx * P.ry;
    uint64_t ns = 1;
    for (int k = 2; k < t.ncols; ++k) {
        ns *= t.card[k];
        if (ns * P.rxy > kMaxCells) {
            P.err = kDevTableTooLarge;
            ns = 1;
            break;
        }
    }
    P.nstrata = (uint32_t)ns;
    P.T = P.rxy * P.nstrata;
    P.df = (int64_t)(P.rx - 1) * (int64_t)(P.ry - 1) * (int64_t)P.nstrata;
    const uint32_t W = (uint32_t)tile.lds_words;
    const uint32_t per_stratum = P.rxy + P.rx + P.ry + 1;  // table + marginals
    uint32_t zc = W / per_stratum;
    if (zc == 0) {
        P.err = kDevTableTooLarge;
        zc = 1;
    }
    if (zc > P.nstrata) zc = P.nstrata;
    P.zc_per = zc;
    P.nchunks = (P.nstrata + zc - 1) / zc;
    P.logR = 0;
    if (P.nchunks == 1) {
        // Replicate while the replicated table still fits next to the reduced one
        // and the zero/reduce work stays small against the m increments.
        const uint32_t marg = (P.rx + P.ry + 1) * P.nstrata;
        const int64_t m = t.m;
        while (P.logR < tile.max_rep_log2) {
            const uint64_t R2 = 2ull << P.logR;
            if ((uint64_t)P.T * R2 + P.T + marg > W) break;
            if ((int64_t)(P.T * R2) * 4 > m) break;
            ++P.logR;
        }
    }
    return P;
}

// Counts, marginals and the G^2 sum of one test over all its chunks in
// precision Real.  Leaves the last chunk's table and marginals in LDS at
// *tab_out / rows / cols / strata.  When gtab is not null the exact counts
// are also written there (cell layout of the table).
template <typename Real>
__device__ inline double table_pass(TestSh &t, const Plan &P, uint32_t *lds, uint32_t *gtab,
                                    const uint32_t **tab_out) {
    Real part = 0;
    const uint32_t *tab = lds;
    for (uint32_t c = 0; c < P.nchunks; ++c) {
        const uint32_t z0 = c * P.zc_per;
        const uint32_t Zc = min(P.zc_per, P.nstrata - z0);
        const uint32_t Tc = P.rxy * Zc;
        const int logR = P.logR;
        uint32_t *rep_tab = lds;
        uint32_t *red = (logR > 0) ? lds + (Tc << logR) : lds;
        uint32_t *rows = red + Tc;
        uint32_t *cols = rows + P.rx * Zc;
        uint32_t *strata = cols + P.ry * Zc;
        for (uint32_t i = threadIdx.x; i < (Tc << logR); i += kWG) rep_tab[i] = 0u;
        __syncthreads();
        count_samples(t, rep_tab, P.rxy * z0, Tc, logR, 0, t.m);
        __syncthreads();
        if (logR > 0) {
            reduce_replicas(rep_tab, red, Tc, logR);
            __syncthreads();
        }
        if (gtab)
            for (uint32_t i = threadIdx.x; i < Tc; i += kWG) gtab[P.rxy * z0 + i] = red[i];
        marginals(red, rows, cols, strata, P.rx, P.ry, Zc);
        part += g2_partial<Real>(red, rows, cols, strata, P.rx, P.ry, Zc);
        tab = red;
        if (c + 1 < P.nchunks) __syncthreads();
    }
    *tab_out = tab;
    const Real s = wg_sum(part, t);
    return 2.0 * (double)s;
}

// FP64 G^2 from a table and marginals still resident in LDS.
__device__ inline double g2_fp64_resident(TestSh &t, const Plan &P, const uint32_t *tab) {
    const uint32_t Zc = P.nstrata;
    const uint32_t *rows = tab + P.rxy * Zc;
    const uint32_t *cols = rows + P.rx * Zc;
    const uint32_t *strata = cols + P.ry * Zc;
    const double part = g2_partial<double>(tab, rows, cols, strata, P.rx, P.ry, Zc);
    return 2.0 * wg_sum(part, t);
}

// Relative error bound of the FP32 G^2 sum: every summand is non-negative and
// carries a few ulp of error, and each thread adds up to ceil(cells/256) of
// them before a 256-way tree, so the relative error stays below
// (8 + cells/256 + 8) * 2^-24 < 1e-5 for tables up to 2^14 cells per pass.
__device__ inline double fp32_g2_rel_bound(const Plan &P) {
    const double per_thread = (double)(P.rxy * P.zc_per) / (double)kWG + 1.0;
    return (16.0 + per_thread) * 5.96e-8 * (double)P.nchunks + 1e-6;
}

// Runs one complete test with the description in t (all threads of the
// workgroup, uniform control flow).  alpha drives the decision; gtab (may be
// null) receives the exact table.
__device__ inline TestOut run_test(TestSh &t, uint32_t *lds, const Tile &tile, double alpha,
                                   uint32_t *gtab) {
    TestOut o;
    o.flags = 0;
    const Plan P = make_plan(t, tile);
    o.err = P.err;
    o.df = P.df;
    if (P.err != kDevOk) {
        o.g2 = 0.0;
        o.p = 1.0;
        return o;
    }
    const uint32_t *tab = nullptr;
    double g2 = tile.fp64 ? table_pass<double>(t, P, lds, gtab, &tab)
                          : table_pass<float>(t, P, lds, gtab, &tab);
    // The chi-square tail is evaluated by one lane and broadcast.
    if (threadIdx.x == 0) {
        double p = chi2_upper(P.df, g2);
        int recheck = 0;
        if (!tile.fp64 && P.df > 0) {
            const double gap = fabs(p - alpha);
            const double a = 0.5 * (double)P.df, x = 0.5 * g2;
            const double dp = gamma_density(a, x) * x * fp32_g2_rel_bound(P);
            recheck = (gap < tile.band) || (gap < 4.0 * dp);
        }
        t.bcast_d[0] = p;
        t.bcast_i[0] = recheck;
    }
    __syncthreads();
    double p = t.bcast_d[0];
    const int recheck = t.bcast_i[0];
    __syncthreads();
    if (recheck) {
        // FP64 re-evaluation: from the resident table when the test fitted in
        // one pass, otherwise by recounting.
        if (P.nchunks == 1) {
            g2 = g2_fp64_resident(t, P, tab);
        } else {
            g2 = table_pass<double>(t, P, lds, nullptr, &tab);
        }
        if (threadIdx.x == 0) t.bcast_d[1] = chi2_upper(P.df, g2);
        __syncthreads();
        p = t.bcast_d[1];
        __syncthreads();
        o.flags |= 2;
    }
    o.g2 = g2;
    o.p = p;
    if (p > alpha) o.flags |= 1;
    return o;
}

}  // namespace bns
