// Device-side building blocks of one G^2 conditional-independence test on
// gfx950: LDS-histogram counting of the contingency table, marginals, the
// G^2 log-sum, the FP64 chi-square tail and the FP64 re-check.
//
// Definitions followed (Jiang, Wen, Mian, Section III-B): N_xyz counts the
// samples with X = x, Y = y, Z = z; E_xyz = N_x+z N_+yz / N_++z;
// G^2 = 2 sum N ln(N / E); p from the chi-square distribution with
// (r_X - 1)(r_Y - 1) prod r_Z degrees of freedom; independence iff p > alpha.
//
// A test is run by a group of lanes (Grp): one wave64, or a whole workgroup
// when one test must be finished by many lanes.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bns_internal.h"

#define BNS_INLINE __device__ __forceinline__

namespace bns {

// ---------------------------------------------------------------------------
// Per-test description staged in LDS (one per group).
// ---------------------------------------------------------------------------
struct TestSh {
    const uint8_t *col[kMaxCols];  // x, y, z_1..z_d columns
    uint32_t card[kMaxCols];
    uint32_t mult[kMaxCols];       // cell stride of each column: 1, r_x, r_x r_y, ...
    int32_t ncols;                 // d + 2
    int64_t m;                     // samples
    double red_d[kWaves];
    float red_f[kWaves];
    double bcast_d[2];
    int32_t bcast_i[2];
};

struct TestOut {
    double g2;
    double p;
    int64_t df;
    int32_t flags;   // bit 0 independent, bit 1 rechecked
    int32_t err;     // DevError
    // verification (run_test<true>): the first-round statistic, its FP64
    // value, and whether the first round's decision differs from FP64's
    double g2_first;
    double g2_ref;
    int32_t flip;
};

// ---------------------------------------------------------------------------
// Groups.  Reductions use a fixed order and broadcast lane 0's result, so
// every lane sees the same, run-to-run deterministic value.
// ---------------------------------------------------------------------------
// Values uniform across a wave (read from LDS by every lane) moved to scalar
// registers, which keeps the per-test state out of the vector register file.
BNS_INLINE uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
BNS_INLINE int32_t uni(int32_t v) { return (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)v); }
BNS_INLINE uint64_t uni(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
BNS_INLINE int64_t uni(int64_t v) { return (int64_t)uni((uint64_t)v); }
BNS_INLINE unsigned long long uni(unsigned long long v) { return (unsigned long long)uni((uint64_t)v); }
BNS_INLINE long long uni(long long v) { return (long long)uni((uint64_t)v); }
BNS_INLINE double uni(double v) { return __builtin_bit_cast(double, uni(__builtin_bit_cast(uint64_t, v))); }
template <typename T>
BNS_INLINE T *uni(T *p) { return (T *)uni((uint64_t)p); }

template <typename T>
BNS_INLINE T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return __shfl(v, 0, 64);
}

// A group of lanes running one test: a wave (block == false; several
// independent tests per workgroup, no workgroup barriers) or the whole
// workgroup (block == true).  The choice is uniform over the group, so the
// branches below never diverge.
struct Grp {
    int rank;
    int size;
    bool block;
    BNS_INLINE static Grp wave() { return Grp{(int)(threadIdx.x & 63), 64, false}; }
    BNS_INLINE static Grp workgroup() { return Grp{(int)threadIdx.x, kWG, true}; }
    BNS_INLINE void sync() const {
        if (block) {
            __syncthreads();
        } else {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    BNS_INLINE double sum(double v, TestSh &t) const {
        v = wave_sum(v);
        if (!block) return v;
        if ((threadIdx.x & 63) == 0) t.red_d[threadIdx.x >> 6] = v;
        __syncthreads();
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) s += t.red_d[w];
        __syncthreads();
        return s;
    }
    // Lane 0's value to every lane of the group.
    BNS_INLINE uint32_t bcast(uint32_t v, TestSh &t) const {
        if (!block) return __shfl(v, 0, 64);
        if (threadIdx.x == 0) t.bcast_i[0] = (int32_t)v;
        __syncthreads();
        v = (uint32_t)t.bcast_i[0];
        __syncthreads();
        return v;
    }
    BNS_INLINE float sum(float v, TestSh &t) const {
        v = wave_sum(v);
        if (!block) return v;
        if ((threadIdx.x & 63) == 0) t.red_f[threadIdx.x >> 6] = v;
        __syncthreads();
        float s = 0.0f;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) s += t.red_f[w];
        __syncthreads();
        return s;
    }
};

// Exact quotient i / d for i < 2^24 via a float reciprocal and one correction.
BNS_INLINE uint32_t fast_div(uint32_t i, uint32_t d, float inv) {
    uint32_t q = (uint32_t)((float)i * inv);
    if (q * d > i) {
        --q;
    } else if ((q + 1) * d <= i) {
        ++q;
    }
    return q;
}

// ---------------------------------------------------------------------------
// Chi-square upper tail in FP64: p = Q(a, x) with a = df/2, x = G^2/2, and
// the Gamma(a, 1) density at x (the slope of Q, used to propagate G^2 error
// bounds), evaluated by all 64 lanes of a wave together; every lane returns
// the same values.
//
// df <= 128 uses the closed forms for integer and half-integer a:
//   a = n:       Q = e^-x sum_{k<n} x^k / k!
//   a = n + 1/2: Q = erfc(sqrt x) + e^-x sum_{k<n} x^(k+1/2) / Gamma(k + 3/2)
// whose terms are formed as a prefix product across lanes (term_k =
// term_{k-1} * x / (k or k + 1/2)).  All summands are positive.
// Larger df: for x below a + 1 + 3 sqrt(a) the lower regularised gamma is
// summed from its power series P = x^a e^-x / Gamma(a+1) sum_k x^k /
// ((a+1)...(a+k)), lane l taking terms [lK, lK + K) from a start formed with
// lgamma; p = 1 - P.  Above it, Legendre's continued fraction for Gamma(a, x)
// (modified Lentz) gives Q directly.
// ---------------------------------------------------------------------------
struct Tail {
    double p;
    double dens;
};

// Large df (> 128): series or continued fraction, out of line (rare).
static __device__ __noinline__ Tail chi2_tail_large(int64_t df, double x) {
    Tail r;
    const int lane = threadIdx.x & 63;
    const double a = 0.5 * (double)df;
    const double lx = log(x);
    r.dens = exp((a - 1.0) * lx - x - lgamma(a));
    if (x < a + 1.0 + 3.0 * sqrt(a)) {
        const double need = fmax(x - a, 0.0) + 10.0 * sqrt(a + x + 1.0) + 40.0;
        const int K = (int)ceil(need / 64.0);
        const double lg1 = lgamma(a + 1.0);
        const double k0 = (double)lane * (double)K;
        double term = exp(k0 * lx - (lgamma(a + 1.0 + k0) - lg1));
        double s = 0.0;
        for (int j = 0; j < K; ++j) {
            s += term;
            term *= x / (a + 1.0 + k0 + (double)j);
        }
        const double tot = wave_sum(s);
        const double lower = exp(a * lx - x - lg1) * tot;
        r.p = lower >= 1.0 ? 0.0 : 1.0 - lower;
        return r;
    }
    const double fpmin = 1e-300;
    double bk = x + 1.0 - a;
    double C = 1.0 / fpmin;
    double D = 1.0 / bk;
    double H = D;
    for (int k = 1; k < 100000; ++k) {
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
    r.p = exp(a * lx - x - lgamma(a)) * H;
    return r;
}

static __device__ __noinline__ Tail chi2_tail_wave(int64_t df, double g2) {
    Tail r;
    r.p = 1.0;
    r.dens = 0.0;
    if (df <= 0) return r;
    const double x = 0.5 * g2;
    if (!(x > 0.0)) return r;
    if (df > 128) return chi2_tail_large(df, x);
    if (x > 700.0) {  // e^-x underflows; the tail is below 1e-200
        r.p = 0.0;
        return r;
    }
    const int lane = threadIdx.x & 63;
    const double pi = 3.141592653589793;
    const int n = (int)(df >> 1);
    const bool odd = (df & 1) != 0;
    double f;
    if (lane == 0) f = odd ? 2.0 * sqrt(x / pi) : 1.0;
    else f = x / ((double)lane + (odd ? 0.5 : 0.0));
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double o = __shfl_up(f, off, 64);
        if (lane >= off) f *= o;
    }
    const double S = wave_sum((lane < n) ? f : 0.0);
    const double last = __shfl(f, n > 0 ? n - 1 : 0, 64);
    const double ex = exp(-x);
    if (odd) {
        r.p = erfc(sqrt(x)) + ex * S;
        r.dens = (n > 0) ? ex * last : ex / sqrt(pi * x);
    } else {
        r.p = ex * S;
        r.dens = ex * last;
    }
    if (r.p > 1.0) r.p = 1.0;
    return r;
}

// The same upper tail evaluated by one lane alone (each lane its own df and
// statistic; no lane exchange): for df <= 128 the closed forms above with the
// terms formed one after another; beyond, the power series of the lower
// function (x below a + 1 + 3 sqrt a) or Legendre's continued fraction by the
// modified Lentz method (Numerical Recipes, 6.2), both run to convergence.
[[maybe_unused]] static __device__ double chi2_tail_lane(int64_t df, double g2) {
    if (df <= 0) return 1.0;
    const double x = 0.5 * g2;
    if (!(x > 0.0)) return 1.0;
    const double pi = 3.141592653589793;
    if (df <= 128) {
        if (x > 700.0) return 0.0;  // e^-x underflows; the tail is below 1e-200
        const int n = (int)(df >> 1);
        const bool odd = (df & 1) != 0;
        const double h = odd ? 0.5 : 0.0;
        double term = odd ? 2.0 * sqrt(x / pi) : 1.0;  // x^(k+h) / Gamma(k+h+1) at k = 0
        double S = 0.0;
        for (int k = 0; k < n; ++k) {
            S += term;
            term *= x / ((double)(k + 1) + h);
        }
        const double p = (odd ? erfc(sqrt(x)) : 0.0) + exp(-x) * S;
        return p > 1.0 ? 1.0 : p;
    }
    const double a = 0.5 * (double)df;
    const double lx = log(x);
    if (x < a + 1.0 + 3.0 * sqrt(a)) {
        double term = 1.0, sum = 1.0;
        for (int k = 1; k < 1000000; ++k) {
            term *= x / (a + (double)k);
            sum += term;
            if (term < sum * 1e-17) break;
        }
        const double lower = exp(a * lx - x - lgamma(a + 1.0)) * sum;
        return lower >= 1.0 ? 0.0 : 1.0 - lower;
    }
    const double fpmin = 1e-300;
    double bk = x + 1.0 - a, C = 1.0 / fpmin, D = 1.0 / bk, H = D;
    for (int k = 1; k < 1000000; ++k) {
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
    return exp(a * lx - x - lgamma(a)) * H;
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
BNS_INLINE Real g2_half_term_exact(uint32_t N, uint32_t nxz, uint32_t nyz, uint32_t nzz) {
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

template <typename Real>
BNS_INLINE Real g2_half_term(uint32_t N, uint32_t nxz, uint32_t nyz, uint32_t nzz) {
    return g2_half_term_exact<Real>(N, nxz, nyz, nzz);
}

// FP32 form with short arithmetic: a and b are formed exactly in FP64 while
// both stay below 2^53, so a - b carries no cancellation error and t has a
// few ulp of relative error; quotients use the hardware reciprocal and the
// logarithm the hardware log2 (about 1 ulp each).
template <>
BNS_INLINE float g2_half_term<float>(uint32_t N, uint32_t nxz, uint32_t nyz, uint32_t nzz) {
    if (N == 0) return (float)nxz * (float)nyz * __builtin_amdgcn_rcpf((float)nzz);
    const double a = (double)N * (double)nzz;
    const double b = (double)nxz * (double)nyz;
    if (a >= 9007199254740992.0 || b >= 9007199254740992.0) return g2_half_term_exact<float>(N, nxz, nyz, nzz);
    const float t = (float)(a - b) * __builtin_amdgcn_rcpf((float)(a + b));
    if (fabsf(t) <= TermCfg<float>::tau) {
        const float u = t * t;
        float sr = 1.0f / (float)(2 * TermCfg<float>::terms + 1);
#pragma unroll
        for (int k = TermCfg<float>::terms - 1; k >= 1; --k) sr = sr * u + 1.0f / (float)(2 * k + 1);
        return (float)N * (2.0f * u * __builtin_amdgcn_rcpf(1.0f + t) + 2.0f * t * u * sr);
    }
    const float w = (float)b * __builtin_amdgcn_rcpf((float)a);
    return (float)N * (w - 1.0f - __logf(w));
}

// ---------------------------------------------------------------------------
// One cell's Pearson term (N - E)^2 / E (the alternative statistic of Section
// II on the same table), E = N_x+z N_+yz / N_++z, written with a = N N_++z and
// b = N_x+z N_+yz (exact integers) as (a - b)^2 / (N_++z b).  Cells with E = 0
// (then also N = 0) contribute 0.  Every term is non-negative.
// ---------------------------------------------------------------------------
template <typename Real>
BNS_INLINE Real x2_term(uint32_t N, uint32_t nxz, uint32_t nyz, uint32_t nzz) {
    const uint64_t b = (uint64_t)nxz * nyz;
    if (b == 0) return (Real)0;
    const uint64_t a = (uint64_t)N * nzz;
    const double dd = (double)((int64_t)a - (int64_t)b);  // exact below 2^53
    const Real d = (Real)dd;
    return (d / (Real)b) * (d / (Real)nzz);
}

template <>
BNS_INLINE float x2_term<float>(uint32_t N, uint32_t nxz, uint32_t nyz, uint32_t nzz) {
    const uint64_t b = (uint64_t)nxz * nyz;
    if (b == 0) return 0.0f;
    const uint64_t a = (uint64_t)N * nzz;
    const float d = (float)(double)((int64_t)a - (int64_t)b);
    return (d * __builtin_amdgcn_rcpf((float)b)) * (d * __builtin_amdgcn_rcpf((float)nzz));
}

// ---------------------------------------------------------------------------
// Counting (step (i) of Section IV-A) into an LDS table.
//
// Columns are uint8, read 16 samples per lane per column with coalesced
// 16-byte loads.  Cell of a sample: sum_k value_k * mult_k.  The table is
// replicated 2^logR times, interleaved per cell (replica = low lane bits), so
// lanes hitting the same cell usually hit different LDS words and banks.
// kChunk: only cells in [cbase, cbase + Tc) are counted (z-range passes of
// tables larger than the LDS slice); other samples go to per-lane spill
// words at `trash`, which keeps the increments unconditional.
// ---------------------------------------------------------------------------
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

BNS_INLINE uint32_t byte_of(const u32x4 &v, int b) {
    const uint32_t w = (b < 4) ? v.x : (b < 8) ? v.y : (b < 12) ? v.z : v.w;
    return (w >> (8 * (b & 3))) & 0xffu;
}

// Global-memory view of a column pointer that is uniform across the wave:
// kept in scalar registers, addressed with a 32-bit per-lane offset.
typedef __attribute__((address_space(1))) const u32x4 gvec4;
typedef __attribute__((address_space(1))) const uint32_t gword;

BNS_INLINE const gvec4 *uniform_col(const uint8_t *p) {
    const uint64_t a = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return (const gvec4 *)(((uint64_t)hi << 32) | lo);
}

// LDS byte offset of a pointer into LDS, and an increment of the LDS word at
// a byte offset.
typedef __attribute__((address_space(3))) uint32_t lds_u32;
BNS_INLINE uint32_t lds_offset(const uint32_t *p) { return (uint32_t)(uintptr_t)(const lds_u32 *)p; }
BNS_INLINE void lds_inc(uint32_t byte_off) {
    __atomic_fetch_add((lds_u32 *)(uintptr_t)byte_off, 1u, __ATOMIC_RELAXED);
}

// Two samples per register: bytes 0 and 2 (or 1 and 3) of a column word are
// moved into the two 16-bit halves, and one 24-bit multiply-add per column
// advances both samples' LDS byte addresses, base + 4 (R cell + replica).
// mul4[k] = 4 R mult_k and base2 holds base + 4 replica in both halves;
// every address stays below 2^16, so the halves never carry into each other.
// NC + 1 vector operations per sample instead of 2 NC + 1.
BNS_INLINE uint32_t mad24(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t d;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(d) : "v"(a), "s"(b), "v"(c));
    return d;
}

template <int NC>
BNS_INLINE void count16_packed(const u32x4 (&v)[NC], const uint32_t (&mul4)[NC], uint32_t base2) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        uint32_t lo = base2, hi = base2;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const uint32_t w = v[k][j];
            lo = mad24(__builtin_amdgcn_perm(0u, w, 0x0c020c00u), mul4[k], lo);  // samples 0, 2
            hi = mad24(__builtin_amdgcn_perm(0u, w, 0x0c030c01u), mul4[k], hi);  // samples 1, 3
        }
        lds_inc(lo & 0xffffu);
        lds_inc(lo >> 16);
        lds_inc(hi & 0xffffu);
        lds_inc(hi >> 16);
    }
}

// Single-pass counting of the groups of 16 samples [q0, q1) into a
// replicated table whose byte addresses lie below 2^16.
template <int NC>
BNS_INLINE void count_packed(const TestSh &t, uint32_t *tab, int logR, int64_t q0, int64_t q1,
                             int rank, int S) {
    constexpr int U = (NC <= 3) ? 4 : 2;
    const uint32_t rep = (uint32_t)rank & ((1u << logR) - 1u);
    const uint32_t b = lds_offset(tab) + 4u * rep;
    const uint32_t base2 = b | (b << 16);
    const gvec4 *cp[NC];
    uint32_t mul4[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        cp[k] = uniform_col(t.col[k]) + q0;
        mul4[k] = __builtin_amdgcn_readfirstlane(t.mult[k] << (logR + 2));
    }
    const uint32_t n = (uint32_t)(q1 - q0);
    const uint32_t us = (uint32_t)S;
    uint32_t i = (uint32_t)rank;
    for (; i + (U - 1) * us < n; i += U * us) {
        u32x4 v[U][NC];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < NC; ++k) v[u][k] = cp[k][i + u * us];
#pragma unroll
        for (int u = 0; u < U; ++u) count16_packed<NC>(v[u], mul4, base2);
    }
    for (; i < n; i += us) {
        u32x4 v[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) v[k] = cp[k][i];
        count16_packed<NC>(v, mul4, base2);
    }
}

template <int NC, bool kChunk>
BNS_INLINE void count16(const u32x4 (&v)[NC], const uint32_t (&mul)[NC], uint32_t *tab,
                        uint32_t cbase, uint32_t Tc, uint32_t trash, int logR, uint32_t rep,
                        uint32_t spill) {
#pragma unroll
    for (int b = 0; b < 16; ++b) {
        uint32_t cell = byte_of(v[0], b);
#pragma unroll
        for (int k = 1; k < NC; ++k) cell += __umul24(byte_of(v[k], b), mul[k]);
        uint32_t addr;
        if (kChunk) {
            const uint32_t idx = cell - cbase;
            addr = (idx < Tc) ? ((idx << logR) | rep) : (trash + spill);
        } else {
            addr = (cell << logR) | rep;
        }
        atomicAdd(&tab[addr], 1u);
    }
}

// Groups of 16 samples [q0, q1), lane `rank` of S taking every S-th group.
template <int NC, bool kChunk>
BNS_INLINE void count_fixed(const TestSh &t, uint32_t *tab, uint32_t cbase, uint32_t Tc,
                            uint32_t trash, int logR, int64_t q0, int64_t q1, int rank, int S) {
    // groups of 16 samples per lane kept in flight per iteration
    constexpr int U = (NC <= 3) ? 4 : 2;
    const uint32_t rep = (uint32_t)rank & ((1u << logR) - 1u);
    const uint32_t spill = (uint32_t)rank;
    const gvec4 *cp[NC];
    uint32_t mul[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        cp[k] = uniform_col(t.col[k]) + q0;
        mul[k] = __builtin_amdgcn_readfirstlane(t.mult[k]);
    }
    // sample groups are < 2^27, so 32-bit group indices suffice
    const uint32_t n = (uint32_t)(q1 - q0);
    const uint32_t us = (uint32_t)S;
    uint32_t i = (uint32_t)rank;
    for (; i + (U - 1) * us < n; i += U * us) {
        u32x4 v[U][NC];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < NC; ++k) v[u][k] = cp[k][i + u * us];
#pragma unroll
        for (int u = 0; u < U; ++u)
            count16<NC, kChunk>(v[u], mul, tab, cbase, Tc, trash, logR, rep, spill);
    }
    for (; i < n; i += us) {
        u32x4 v[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) v[k] = cp[k][i];
        count16<NC, kChunk>(v, mul, tab, cbase, Tc, trash, logR, rep, spill);
    }
}

template <bool kChunk>
BNS_INLINE void count_generic(const TestSh &t, uint32_t *tab, uint32_t cbase, uint32_t Tc,
                              uint32_t trash, int logR, int64_t q0, int64_t q1, int rank, int S) {
    const uint32_t rep = (uint32_t)rank & ((1u << logR) - 1u);
    const uint32_t spill = (uint32_t)rank;
    const int nc = t.ncols;
    for (int64_t q = q0 + rank; q < q1; q += S) {
        uint32_t cell[16];
        {
            const u32x4 v = uniform_col(t.col[0])[q];
#pragma unroll
            for (int b = 0; b < 16; ++b) cell[b] = byte_of(v, b);
        }
        for (int k = 1; k < nc; ++k) {
            const u32x4 v = uniform_col(t.col[k])[q];
            const uint32_t mk = __builtin_amdgcn_readfirstlane(t.mult[k]);
#pragma unroll
            for (int b = 0; b < 16; ++b) cell[b] += __umul24(byte_of(v, b), mk);
        }
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            uint32_t addr;
            if (kChunk) {
                const uint32_t idx = cell[b] - cbase;
                addr = (idx < Tc) ? ((idx << logR) | rep) : (trash + spill);
            } else {
                addr = (cell[b] << logR) | rep;
            }
            atomicAdd(&tab[addr], 1u);
        }
    }
}

// Samples [s0, s1) one byte at a time (the ragged tail after the 16-sample groups).
template <bool kChunk>
BNS_INLINE void count_tail(const TestSh &t, uint32_t *tab, uint32_t cbase, uint32_t Tc,
                           uint32_t trash, int logR, int64_t s0, int64_t s1, int rank, int S) {
    const uint32_t rep = (uint32_t)rank & ((1u << logR) - 1u);
    for (int64_t s = s0 + rank; s < s1; s += S) {
        uint32_t cell = t.col[0][s];
        for (int k = 1; k < t.ncols; ++k) cell += __umul24((uint32_t)t.col[k][s], t.mult[k]);
        uint32_t addr;
        if (kChunk) {
            const uint32_t idx = cell - cbase;
            addr = (idx < Tc) ? ((idx << logR) | rep) : (trash + (uint32_t)rank);
        } else {
            addr = (cell << logR) | rep;
        }
        atomicAdd(&tab[addr], 1u);
    }
}

// Counts samples [s0, s1) (s0 a multiple of 16) with the S lanes of a group.
// kNcMax: the most columns the instance specialises (tests of more columns
// take the generic loop); an instance for shallow depths leaves out the wide
// unrolled loops and the registers they hold.
template <bool kChunk, int kNcMax = kMaxCols>
BNS_INLINE void count_range(const TestSh &t, uint32_t *tab, uint32_t cbase, uint32_t Tc,
                            uint32_t trash, int logR, int64_t s0, int64_t s1, int rank, int S) {
    const int64_t q0 = s0 >> 4, q1 = s1 >> 4;
    const int nc = uni(t.ncols);
    if (!kChunk) {
        // packed path when every byte address of the replicated table fits 16 bits
        const bool packed = nc <= 6 && (uint64_t)lds_offset(tab) + 4ull * ((uint64_t)Tc << logR) <= 65536ull;
        if (packed) {
            switch (nc) {
                case 2: count_packed<2>(t, tab, logR, q0, q1, rank, S); break;
                case 3: count_packed<3>(t, tab, logR, q0, q1, rank, S); break;
                case 4: count_packed<4>(t, tab, logR, q0, q1, rank, S); break;
                default:
                    if constexpr (kNcMax >= 6) {
                        if (nc == 5) count_packed<5>(t, tab, logR, q0, q1, rank, S);
                        else count_packed<6>(t, tab, logR, q0, q1, rank, S);
                    } else {
                        count_generic<false>(t, tab, cbase, Tc, trash, logR, q0, q1, rank, S);
                    }
                    break;
            }
        } else {
            count_generic<false>(t, tab, cbase, Tc, trash, logR, q0, q1, rank, S);
        }
    } else {
        switch (nc) {
            case 2: count_fixed<2, true>(t, tab, cbase, Tc, trash, logR, q0, q1, rank, S); break;
            case 3: count_fixed<3, true>(t, tab, cbase, Tc, trash, logR, q0, q1, rank, S); break;
            case 4: count_fixed<4, true>(t, tab, cbase, Tc, trash, logR, q0, q1, rank, S); break;
            default:
                if constexpr (kNcMax >= 6) {
                    if (nc == 5) {
                        count_fixed<5, true>(t, tab, cbase, Tc, trash, logR, q0, q1, rank, S);
                        break;
                    }
                    if (nc == 6) {
                        count_fixed<6, true>(t, tab, cbase, Tc, trash, logR, q0, q1, rank, S);
                        break;
                    }
                }
                count_generic<true>(t, tab, cbase, Tc, trash, logR, q0, q1, rank, S);
                break;
        }
    }
    if ((q1 << 4) < s1) count_tail<kChunk>(t, tab, cbase, Tc, trash, logR, q1 << 4, s1, rank, S);
}

// Sums the 2^logR interleaved replicas of each cell: out[c] = sum_r rep[c * R + r].
// Lane c starts at replica c mod R, so the lanes of a wave read R (up to 64)
// different banks at every step.
BNS_INLINE void reduce_replicas(const uint32_t *rep_tab, uint32_t *out, uint32_t Tc, int logR,
                                int rank, int S) {
    const uint32_t R = 1u << logR, mask = R - 1u;
    // L = 2^lgL lanes per cell when the cells leave lanes idle: each sums
    // R / L (at least 4) replicas and the L partial sums (consecutive lanes
    // of one wave) are combined with lane exchanges.
    int lgL = 0;
    while (lgL < 6 && (Tc << (lgL + 1)) <= (uint32_t)S && (8u << lgL) <= R) ++lgL;
    const uint32_t span = R >> lgL;
    const uint32_t j = (uint32_t)rank & ((1u << lgL) - 1u);
    for (uint32_t c0 = 0; c0 < Tc; c0 += (uint32_t)S >> lgL) {
        const uint32_t c = c0 + ((uint32_t)rank >> lgL);
        uint32_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        if (c < Tc) {
            // (replica r + c of cell c: neighbouring cells start on different banks)
            const uint32_t *p = rep_tab + (c << logR);
            uint32_t r = j * span;
            const uint32_t r1 = r + span;
            for (; r + 4 <= r1; r += 4) {
                s0 += p[(r + c) & mask];
                s1 += p[(r + 1 + c) & mask];
                s2 += p[(r + 2 + c) & mask];
                s3 += p[(r + 3 + c) & mask];
            }
            for (; r < r1; ++r) s0 += p[(r + c) & mask];
        }
        uint32_t sum = (s0 + s1) + (s2 + s3);
        for (int off = 1; off < (1 << lgL); off <<= 1) sum += (uint32_t)__shfl_xor((int)sum, off, 64);
        if (c < Tc && j == 0) out[c] = sum;
    }
}

// Marginal tables of a chunk of Zc strata (step (ii) of Section IV-A):
// rows[x + rx z] = N_x+z, cols[y + ry z] = N_+yz, strata[z] = N_++z.
BNS_INLINE void marginals(const Grp &g, const uint32_t *tab, uint32_t *rows, uint32_t *cols,
                          uint32_t *strata, uint32_t rx, uint32_t ry, uint32_t Zc) {
    const float inv_rx = 1.0f / (float)rx;
    const uint32_t nrow = rx * Zc, ncol = ry * Zc;
    for (uint32_t i = g.rank; i < nrow + ncol; i += g.size) {
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
    g.sync();
    for (uint32_t z = g.rank; z < Zc; z += g.size) {
        uint32_t s = 0;
        for (uint32_t yv = 0; yv < ry; ++yv) s += cols[yv + ry * z];
        strata[z] = s;
    }
    g.sync();
}

// This lane's part of the sum of the statistic's cell terms over a chunk
// (g2_half_term for G^2, stat 0; x2_term for X^2, stat 1): one cell per lane
// and step (a table with no more cells than lanes costs one term).
template <typename Real>
BNS_INLINE Real stat_partial(const Grp &g, const uint32_t *tab, const uint32_t *rows,
                             const uint32_t *cols, const uint32_t *strata, uint32_t rx, uint32_t ry,
                             uint32_t Zc, int stat) {
    const float inv_rx = 1.0f / (float)rx, inv_ry = 1.0f / (float)ry;
    const uint32_t T = rx * ry * Zc;
    Real acc = 0;
    for (uint32_t c = g.rank; c < T; c += g.size) {
        const uint32_t rho = fast_div(c, rx, inv_rx);  // y + ry z
        const uint32_t xv = c - rho * rx;
        const uint32_t z = fast_div(rho, ry, inv_ry);
        const uint32_t nzz = strata[z];
        if (nzz == 0) continue;
        if (stat) acc += x2_term<Real>(tab[c], rows[xv + rx * z], cols[rho], nzz);
        else acc += g2_half_term<Real>(tab[c], rows[xv + rx * z], cols[rho], nzz);
    }
    return acc;
}

// This lane's part of the adjusted degrees of freedom of a chunk of strata:
// per stratum with N_++z > 0, (non-empty rows - 1)(non-empty columns - 1).
BNS_INLINE double adj_df_partial(const Grp &g, const uint32_t *rows, const uint32_t *cols,
                                 const uint32_t *strata, uint32_t rx, uint32_t ry, uint32_t Zc) {
    double acc = 0.0;
    for (uint32_t z = g.rank; z < Zc; z += g.size) {
        if (strata[z] == 0) continue;
        uint32_t a = 0, b = 0;
        for (uint32_t xv = 0; xv < rx; ++xv) a += rows[xv + rx * z] > 0u ? 1u : 0u;
        for (uint32_t yv = 0; yv < ry; ++yv) b += cols[yv + ry * z] > 0u ? 1u : 0u;
        acc += (double)(a - 1u) * (double)(b - 1u);
    }
    return acc;
}

// ---------------------------------------------------------------------------
// Pass plan of a test: strata per LDS pass and the replication of the table.
// ---------------------------------------------------------------------------
struct Plan {
    uint32_t rx, ry, rxy;
    uint32_t nstrata;     // prod r_z
    uint32_t T;           // cells
    uint32_t zc_per;      // strata per pass
    uint32_t nchunks;
    int logR;             // replication of single-pass tables
    int64_t df;
    int32_t err;
};

// W: LDS words available to the group; S: lanes in the group; msamp: samples
// the group counts (replication must stay cheap against them); addr_words:
// words of the slice below LDS byte 2^16 (replication stops there so that
// single-pass counting can use 16-bit addresses).
BNS_INLINE Plan make_plan(const TestSh &t, uint32_t W, int max_rep_log2, int S, int64_t msamp,
                          uint32_t addr_words) {
    Plan P;
    P.err = kDevOk;
    P.rx = uni(t.card[0]);
    P.ry = uni(t.card[1]);
    P.rxy = P.rx * P.ry;
    uint64_t ns = 1;
    const int nc = uni(t.ncols);
    for (int k = 2; k < nc; ++k) {
        ns *= uni(t.card[k]);
        if (ns * P.rxy > kMaxCells) {
            P.err = kDevTableTooLarge;
            ns = 1;
            break;
        }
    }
    P.nstrata = (uint32_t)ns;
    P.T = P.rxy * P.nstrata;
    P.df = (int64_t)(P.rx - 1) * (int64_t)(P.ry - 1) * (int64_t)P.nstrata;
    const uint32_t per_stratum = P.rxy + P.rx + P.ry + 1;  // table + marginals
    const uint32_t marg = (P.rx + P.ry + 1) * P.nstrata;
    P.logR = 0;
    if ((uint64_t)P.T + marg <= W) {
        P.zc_per = P.nstrata;
        P.nchunks = 1;
        // Replicate while the replicated table fits next to the reduced one
        // and the zero/reduce work stays small against the increments.
        const int64_t m = msamp;
        while (P.logR < max_rep_log2) {
            const uint64_t R2 = 2ull << P.logR;
            if ((uint64_t)P.T * R2 + P.T + marg > W) break;
            if ((uint64_t)P.T * R2 > addr_words) break;
            if ((int64_t)(P.T * R2) * 4 > m + 16 * S) break;
            ++P.logR;
        }
    } else {
        // Passes over z ranges; S spill words follow the counted cells.
        uint32_t zc = (W > (uint32_t)S) ? (W - (uint32_t)S) / per_stratum : 0;
        if (zc == 0) {
            P.err = kDevTableTooLarge;
            zc = 1;
        }
        if (zc > P.nstrata) zc = P.nstrata;
        P.zc_per = zc;
        P.nchunks = (P.nstrata + zc - 1) / zc;
    }
    return P;
}

// Reads a counter that other workgroups updated with device-scope atomics.
BNS_INLINE uint32_t load_device(const uint32_t *p) {
    return __hip_atomic_load(const_cast<uint32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Where the counts of a pass come from and where they go.
struct Src {
    const uint32_t *gsrc;  // non-null: read the table from here (merged chunks of a split test)
    uint32_t *gdst;        // non-null: add the counted table to here, no G^2
    int64_t s0, s1;        // samples counted (s0 a multiple of 16)
};

// Counts, marginals and the G^2 sum of one test over all its passes (G^2 in
// FP64 when fp64, else FP32).  Leaves the last pass's table and marginals in
// LDS (returned through *tab_out).  gtab (may be null) receives the counts.
// With src.gsrc the table is read instead of counted (the plan must have no
// replication); with src.gdst the counts of samples [s0, s1) are added to
// src.gdst with device-scope atomics (non-zero cells only) and nothing else
// is computed.
// The statistic is G^2 (stat 0) or X^2 (stat 1); with df_adj the adjusted
// degrees of freedom of the table are summed into *df_adj.
template <int kNcMax = kMaxCols>
BNS_INLINE double table_pass(const Grp &g, TestSh &t, const Plan &P, uint32_t *lds, uint32_t *gtab,
                             const Src &src, bool fp64, const uint32_t **tab_out, int stat,
                             double *df_adj) {
    double part64 = 0.0, dfp = 0.0;
    float part32 = 0.0f;
    const uint32_t *tab = lds;
    const bool chunked = P.nchunks > 1;
    for (uint32_t c = 0; c < P.nchunks; ++c) {
        const uint32_t z0 = c * P.zc_per;
        const uint32_t Zc = min(P.zc_per, P.nstrata - z0);
        const uint32_t Tc = P.rxy * Zc;
        const int logR = P.logR;
        uint32_t *rep_tab = lds;
        // layout: [replicated table | spill words (passes)] [reduced table (R > 1)]
        //         [rows] [cols] [strata]
        const uint32_t head = (Tc << logR) + (chunked ? (uint32_t)g.size : 0u);
        uint32_t *red = (logR > 0) ? lds + head : lds;
        uint32_t *rows = lds + head + (logR > 0 ? Tc : 0u);
        uint32_t *cols = rows + P.rx * Zc;
        uint32_t *strata = cols + P.ry * Zc;
        if (src.gsrc) {
            // sixteen device loads in flight per lane before any is stored
            // (4,096 cells per round trip of a workgroup)
            const uint32_t *gs = src.gsrc + P.rxy * z0;
            for (uint32_t i0 = g.rank; i0 < Tc; i0 += 16u * (uint32_t)g.size) {
                uint32_t v[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const uint32_t i = i0 + (uint32_t)u * (uint32_t)g.size;
                    v[u] = i < Tc ? load_device(gs + i) : 0u;
                }
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const uint32_t i = i0 + (uint32_t)u * (uint32_t)g.size;
                    if (i < Tc) red[i] = v[u];
                }
            }
            g.sync();
        } else {
            for (uint32_t i = g.rank; i < head; i += g.size) rep_tab[i] = 0u;
            g.sync();
            if (chunked)
                count_range<true, kNcMax>(t, rep_tab, P.rxy * z0, Tc, Tc, 0, src.s0, src.s1, g.rank, g.size);
            else
                count_range<false, kNcMax>(t, rep_tab, 0, Tc, 0, logR, src.s0, src.s1, g.rank, g.size);
            g.sync();
            if (logR > 0) {
                reduce_replicas(rep_tab, red, Tc, logR, g.rank, g.size);
                g.sync();
            }
        }
        if (src.gdst) {
            // Adds in the returning form: once an add's old value has arrived
            // the add has been performed at the device's coherence point, so
            // the group's wait for its memory operations, before the chunk
            // counter is incremented, orders every add of the chunk before the
            // increment.  (The returned values are kept live; counts stay
            // below 2^31, so their union is never all ones.)
            uint32_t *dst = src.gdst + P.rxy * z0;
            uint32_t seen = 0u;
            for (uint32_t i = g.rank; i < Tc; i += g.size) {
                const uint32_t v = red[i];
                if (v) seen |= __hip_atomic_fetch_add(dst + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (seen == ~0u) t.bcast_i[1] = 1;
            if (c + 1 < P.nchunks) g.sync();
            continue;
        }
        if (gtab)
            for (uint32_t i = g.rank; i < Tc; i += g.size) gtab[P.rxy * z0 + i] = red[i];
        marginals(g, red, rows, cols, strata, P.rx, P.ry, Zc);
        if (fp64) part64 += stat_partial<double>(g, red, rows, cols, strata, P.rx, P.ry, Zc, stat);
        else part32 += stat_partial<float>(g, red, rows, cols, strata, P.rx, P.ry, Zc, stat);
        if (df_adj) dfp += adj_df_partial(g, rows, cols, strata, P.rx, P.ry, Zc);
        tab = red;
        if (c + 1 < P.nchunks) g.sync();
    }
    *tab_out = tab;
    if (src.gdst) return 0.0;
    if (df_adj) *df_adj = g.sum(dfp, t);
    const double scale = stat ? 1.0 : 2.0;  // G^2 = 2 sum of the half terms
    if (fp64) return scale * g.sum(part64, t);
    return scale * (double)g.sum(part32, t);
}

// FP64 statistic from a single-pass table and marginals still resident in LDS.
BNS_INLINE double stat_fp64_resident(const Grp &g, TestSh &t, const Plan &P, const uint32_t *tab, int stat) {
    const uint32_t Zc = P.nstrata;
    const uint32_t *rows = tab + P.rxy * Zc;
    const uint32_t *cols = rows + P.rx * Zc;
    const uint32_t *strata = cols + P.ry * Zc;
    const double part = stat_partial<double>(g, tab, rows, cols, strata, P.rx, P.ry, Zc, stat);
    return (stat ? 1.0 : 2.0) * g.sum(part, t);
}

// Relative error bound of the FP32 G^2 sum: every summand is non-negative and
// carries at most a few tens of ulp of error (conversions, reciprocals, the
// series or the log2), and each lane adds up to ceil(cells/lanes) of them
// before a tree, so the relative error stays below (32 + cells/lanes) * 2^-24
// per pass.
BNS_INLINE double fp32_g2_rel_bound(const Plan &P, int S) {
    const double per_lane = (double)(P.rxy * P.zc_per) / (double)S + 1.0;
    return (32.0 + per_lane) * 5.96e-8 * (double)P.nchunks + 1e-6;
}

// Tail of the group (chi2_tail_wave needs a whole wave; a workgroup lets its
// first wave evaluate it and broadcasts).
BNS_INLINE Tail group_tail(const Grp &g, int64_t df, double g2, TestSh &t) {
    if (!g.block) return chi2_tail_wave(df, g2);
    Tail r;
    r.p = 0.0;
    r.dens = 0.0;
    if (threadIdx.x < 64) r = chi2_tail_wave(df, g2);
    if (threadIdx.x == 0) {
        t.bcast_d[0] = r.p;
        t.bcast_d[1] = r.dens;
    }
    __syncthreads();
    r.p = t.bcast_d[0];
    r.dens = t.bcast_d[1];
    __syncthreads();
    return r;
}

// Runs one complete test with the description in t (all lanes of the group,
// uniform control flow) in W words of LDS at lds.  alpha drives the decision;
// gtab (may be null) receives the exact table.  src: the samples counted, or
// the merged table of a split test to evaluate, or a merge target (then only
// the chunk [s0, s1) is counted and added there; no G^2, no decision).
// kGeneral: the statistic and df rule come from the tile; otherwise the
// instance is fixed to G^2 with df from the declared cards.
template <bool kVerify = false, bool kGeneral = true, int kNcMax = kMaxCols>
BNS_INLINE TestOut run_test(const Grp &g, TestSh &t, uint32_t *lds, uint32_t W, const Tile &tile,
                            double alpha, uint32_t *gtab, const Src &src) {
    TestOut o;
    o.flags = 0;
    o.g2_first = 0.0;
    o.g2_ref = 0.0;
    o.flip = 0;
    const uint32_t lo = lds_offset(lds);
    const uint32_t addr_words = lo < 65536u ? (65536u - lo) / 4u : 0u;
    const Plan P = make_plan(t, W, src.gsrc ? 0 : tile.max_rep_log2, g.size, src.s1 - src.s0,
                             addr_words);
    o.err = P.err;
    o.df = P.df;
    if (P.err != kDevOk) {
        o.g2 = 0.0;
        o.p = 1.0;
        return o;
    }
    // One counting pass in the requested precision; an FP32 decision close to
    // alpha is re-evaluated in FP64, from the resident table when the test
    // fitted in one pass, otherwise by a second counting pass.
    const uint32_t *tab = nullptr;
    bool fp64 = tile.fp64 != 0;
    const int stat = kGeneral ? tile.stat : 0;
    const bool adj = kGeneral && tile.df_rule != 0;
    double g2 = 0.0, p = 1.0, p_first = 1.0;
    int64_t df = P.df;
    for (int round = 0; round < 2; ++round) {
        double dfa = 0.0;
        g2 = table_pass<kNcMax>(g, t, P, lds, round == 0 ? gtab : nullptr, src, fp64, &tab, stat,
                        adj ? &dfa : nullptr);
        if (src.gdst) {  // merge only: no statistic, no decision
            o.g2 = 0.0;
            o.p = 1.0;
            return o;
        }
        if (adj) df = (int64_t)dfa;
        Tail tl = group_tail(g, df, g2, t);
        p = tl.p;
        if (round == 0) {
            o.g2_first = g2;
            p_first = p;
        }
        if (fp64 || df <= 0) break;
        const double gap = fabs(p - alpha);
        // propagate the FP32 error bound of the statistic through the tail's slope
        const double dp = tl.dens * 0.5 * g2 * fp32_g2_rel_bound(P, g.size);
        if (!(gap < tile.band || gap < 4.0 * dp)) break;
        o.flags |= 2;
        if (P.nchunks > 1) {
            fp64 = true;
            continue;
        }
        g2 = stat_fp64_resident(g, t, P, tab, stat);
        p = group_tail(g, df, g2, t).p;
        break;
    }
    o.df = df;
    o.g2 = g2;
    o.p = p;
    if (p > alpha) o.flags |= 1;
    if (kVerify) {
        // FP64 value of the statistic: the decision's own when it was FP64,
        // else from the table still in LDS (one pass) or by counting again.
        double g64 = g2, p64 = p;
        if (!fp64 && !(o.flags & 2) && df > 0) {
            if (P.nchunks == 1) g64 = stat_fp64_resident(g, t, P, tab, stat);
            else g64 = table_pass<kNcMax>(g, t, P, lds, nullptr, src, true, &tab, stat, nullptr);
            p64 = group_tail(g, df, g64, t).p;
        }
        o.g2_ref = g64;
        o.flip = ((p_first > alpha) != (p64 > alpha)) ? 1 : 0;
    }
    return o;
}

}  // namespace bns
