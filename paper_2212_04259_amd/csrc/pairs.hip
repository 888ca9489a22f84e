// Depth 0 of the skeleton search (Section IV-B: every pair is tested once,
// with no conditioning set) as one dense contraction on gfx950 int8 MFMA.
//
// With one-hot columns A[s][(v, x)] = [X_v(s) = x] (m samples by R = sum of
// the cardinalities), the Gram matrix A^T A holds every pairwise contingency
// table: N_ij[x][y] = (A^T A)[(i, x)][(j, y)], and its diagonal the count of
// each category, which are the marginals N_x+ and N_+y of every pair table.
// The products of 0/1 bytes summed in int32 are exact (m < 2^31).
//
// k_gram: one work item is a T x T tile of the upper triangle of tile blocks
// of one problem's Gram matrix over one chunk of samples; a workgroup (2 x 2
// waves, each a (T/2) x (T/2) block of 32 x 32 MFMA tiles) expands the tile's
// one-hot columns for 64 samples at a time into LDS (double-buffered: the
// global loads of the next step are in flight during the MFMAs of this one)
// and writes its partial tile.
// k_gram_reduce: sums each tile's partials over its problem's chunks.
// k_depth0_pairs: one lane per edge of the depth reads the pair's block of the
// summed tiles, forms the statistic in FP64, its own chi-square tail and the
// decision.
#include <algorithm>

#include "device_ci.h"
#include "gram.h"
#include "kernels.h"

namespace bns {

constexpr int kGramKS = 64;             // samples per pipeline step
constexpr int kGramRow = kGramKS + 16;  // LDS bytes per one-hot column and step
constexpr int kGramQS = kGramKS / 16;   // 16-sample groups per column and step

// c: the search's control block (its done flag, the depth's start stamp), or
// null for the all-pairs entry point.
template <int T>
__global__ __launch_bounds__(kGramWG) void k_gram(PairArgs P, Ctl *c) {
    constexpr int WT = T / 2;              // rows (and columns) of a wave's block
    constexpr int NF = WT / 32;            // 32 x 32 MFMA tiles per side of a wave's block
    constexpr int kTasks = 2 * T * kGramQS;  // (operand, column, 16-sample group) per step
    constexpr int kPer = kTasks / kGramWG;
    static_assert(kPer * kGramWG == kTasks, "tasks split evenly");
    __shared__ __attribute__((aligned(16))) uint8_t lds[2][2 * T * kGramRow];  // [buffer][operand][column][sample]
    __shared__ int quit;
    if (threadIdx.x == 0) {
        quit = c ? c->done : 0;
        if (c && blockIdx.x == 0) {
            c->stats[0].t_start = wall_clock64();
            c->stats[0].mode = 2;  // depth 0 as the pair contraction
            c->stats[0].chunks = 0;
            c->stats[0].chunk_len = P.chunk;
        }
    }
    __syncthreads();
    if (quit) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = w >> 1, wc = w & 1;
    for (int64_t item = blockIdx.x; item < P.items; item += gridDim.x) {
        // work item -> problem, tile (tr <= tc), chunk of samples
        int lo = 0, hi = P.n_gp - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (P.gp[mid].item_base <= item) lo = mid;
            else hi = mid - 1;
        }
        const GramProb gp = P.gp[lo];
        const int64_t rel = item - gp.item_base;
        const int64_t t = rel / gp.nchunks;
        const int kc = (int)(rel - t * gp.nchunks);
        int tr = 0;
        int64_t rem = t;
        while (rem >= gp.nb - tr) {
            rem -= gp.nb - tr;
            ++tr;
        }
        const int tc = tr + (int)rem;
        const bool diag = tr == tc;  // the second operand is the first
        const int64_t s0 = (int64_t)kc * P.chunk;
        const int64_t s1 = min(gp.m, s0 + P.chunk);
        const int nsteps = (int)((s1 - s0 + kGramKS - 1) / kGramKS);
        // this thread's expansion tasks for every step of the item
        const uint8_t *colp[kPer];
        uint32_t plo[kPer], phi[kPer], cat[kPer];
        int dst[kPer];
        bool act[kPer], wide[kPer];
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int id = tid + kGramWG * r;
            const int op = id / (T * kGramQS);
            const int rest = id - op * T * kGramQS;
            const int col = rest / kGramQS, q = rest % kGramQS;
            act[r] = !(diag && op == 1);
            dst[r] = op * T * kGramRow + col * kGramRow + 16 * q;
            const int gcol = (op ? tc : tr) * T + col;
            const int v = P.oh_var[gp.oh_base + gcol];
            const uint32_t cb = P.oh_cat[gp.oh_base + gcol];
            wide[r] = (cb & 0x100u) != 0;
            cat[r] = cb & 0xffu;
            plo[r] = cat[r] < 4 ? 1u << (8 * cat[r]) : 0u;
            phi[r] = (cat[r] >= 4 && cat[r] < 8) ? 1u << (8 * (cat[r] - 4)) : 0u;
            colp[r] = v >= 0 ? gp.data + (int64_t)v * gp.ld + 16 * q : nullptr;
        }
        u32x4 pv[kPer];
        int pn[kPer];
        auto load = [&](int64_t s) {
            // samples left from s (uniform; at most a step and a group matter)
            const int left = (int)min(s1 - s, (int64_t)(kGramKS + 16));
#pragma unroll
            for (int r = 0; r < kPer; ++r) {
                pn[r] = min(16, max(0, left - 16 * ((tid + kGramWG * r) % kGramQS)));
                pv[r] = u32x4{0u, 0u, 0u, 0u};
                // (a global load: a flat one would also count against the
                // LDS counter, and the step's LDS reads would wait for it)
                if (act[r] && colp[r] && pn[r] > 0) pv[r] = *(const gvec4 *)(colp[r] + s);
            }
        };
        auto store = [&](int buf) {
#pragma unroll
            for (int r = 0; r < kPer; ++r) {
                if (!act[r]) continue;
                u32x4 o = u32x4{0u, 0u, 0u, 0u};
                if (colp[r]) o = onehot16(pv[r], plo[r], phi[r], cat[r], wide[r], pn[r]);
                *(u32x4 *)(&lds[buf][dst[r]]) = o;
            }
        };
        v16i acc[NF][NF];
#pragma unroll
        for (int i = 0; i < NF; ++i)
#pragma unroll
            for (int j = 0; j < NF; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;
        load(s0);
        store(0);
        __syncthreads();
        for (int st = 0; st < nsteps; ++st) {
            const int buf = st & 1;
            const bool more = st + 1 < nsteps;
            if (more) load(s0 + (int64_t)(st + 1) * kGramKS);
            const uint8_t *La = &lds[buf][0];
            const uint8_t *Lb = diag ? La : &lds[buf][T * kGramRow];
#pragma unroll
            for (int kk = 0; kk < kGramKS / 32; ++kk) {
                const int koff = 32 * kk + 16 * (lane >> 5);
                v4i af[NF], bf[NF];
#pragma unroll
                for (int i = 0; i < NF; ++i)
                    af[i] = *(const v4i *)(La + (wr * WT + 32 * i + (lane & 31)) * kGramRow + koff);
#pragma unroll
                for (int j = 0; j < NF; ++j)
                    bf[j] = *(const v4i *)(Lb + (wc * WT + 32 * j + (lane & 31)) * kGramRow + koff);
#pragma unroll
                for (int i = 0; i < NF; ++i)
#pragma unroll
                    for (int j = 0; j < NF; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[i], bf[j], acc[i][j], 0, 0, 0);
            }
            if (more) store(buf ^ 1);
            __syncthreads();
        }
        // partial tile of the item: register r of lane l holds row
        // (r % 4) + 4 (l / 32) + 8 (r / 4), column l % 32 of a 32 x 32 tile
        int32_t *out = P.part + item * (int64_t)(T * T);
#pragma unroll
        for (int i = 0; i < NF; ++i)
#pragma unroll
            for (int j = 0; j < NF; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = wr * WT + 32 * i + (r & 3) + 4 * (lane >> 5) + 8 * (r >> 2);
                    const int col = wc * WT + 32 * j + (lane & 31);
                    out[row * T + col] = acc[i][j][r];
                }
    }
}

// Sums each tile's partials over its problem's chunks (coalesced, four
// entries per lane): gram[tile] = sum_k part[item of (tile, k)].
__global__ __launch_bounds__(kWG) void k_gram_reduce(PairArgs P) {
    const int64_t tq = (int64_t)P.T * P.T / 4;  // int4 words per tile
    const int64_t total = P.tiles * tq;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < total; i += (int64_t)gridDim.x * kWG) {
        const int64_t tile = i / tq, w = i - tile * tq;
        int lo = 0, hi = P.n_gp - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (P.gp[mid].tile_base <= tile) lo = mid;
            else hi = mid - 1;
        }
        const GramProb &gp = P.gp[lo];
        const int4 *src = (const int4 *)P.part + (gp.item_base + (tile - gp.tile_base) * gp.nchunks) * tq + w;
        int4 s = src[0];
        for (int k = 1; k < gp.nchunks; ++k) {
            const int4 v = src[(int64_t)k * tq];
            s.x += v.x;
            s.y += v.y;
            s.z += v.z;
            s.w += v.w;
        }
        ((int4 *)P.gram)[i] = s;
    }
}

// Entry (a, b), a <= b, of a problem's Gram matrix.
BNS_INLINE uint32_t gram_entry(const PairArgs &P, const GramProb &gp, int a, int b) {
    const int T = P.T;
    const int ta = a / T, tb = b / T;
    const int64_t ti = (int64_t)ta * gp.nb - (int64_t)ta * (ta - 1) / 2 + (tb - ta);
    return (uint32_t)P.gram[(gp.tile_base + ti) * (int64_t)T * T + (int64_t)(a - ta * T) * T + (b - tb * T)];
}

// Statistic (G^2 or X^2, FP64) and df of the pair of variables whose one-hot
// columns start at oi and oj (oi < oj) with ri and rj categories, over m
// samples: the table is the pair's block of the Gram matrix, the marginals
// N_x+ and N_+y its diagonal entries (the category counts), N_++ = m.
BNS_INLINE void pair_stat(const PairArgs &P, const GramProb &gp, int oi, int oj, int ri, int rj, int64_t m,
                          int stat_kind, bool adj, double &stat, int64_t &df) {
    int na = 0, nb = 0;
    stat = 0.0;
    for (int y = 0; y < rj; ++y) nb += gram_entry(P, gp, oj + y, oj + y) > 0u ? 1 : 0;
    for (int x = 0; x < ri; ++x) {
        const uint32_t nx = gram_entry(P, gp, oi + x, oi + x);  // N_x+
        na += nx > 0u ? 1 : 0;
        for (int y = 0; y < rj; ++y) {
            const uint32_t ny = gram_entry(P, gp, oj + y, oj + y);  // N_+y
            const uint32_t N = gram_entry(P, gp, oi + x, oj + y);
            if (stat_kind) stat += x2_term<double>(N, nx, ny, (uint32_t)m);
            else stat += g2_half_term<double>(N, nx, ny, (uint32_t)m);
        }
    }
    if (!stat_kind) stat *= 2.0;
    df = adj ? (int64_t)(na - 1) * (int64_t)(nb - 1) : (int64_t)(ri - 1) * (int64_t)(rj - 1);
}

// The depth-0 tests of a skeleton search: one lane per edge of the depth.
__global__ __launch_bounds__(kWG) void k_depth0_pairs(DepthArgs A) {
    Ctl *c = A.ctl;
    __shared__ int quit;
    if (threadIdx.x == 0) quit = c->done;
    __syncthreads();
    if (quit) return;
    const PairArgs &P = A.pairs;
    const unsigned long long E = c->n_edges;
    const int lane = threadIdx.x & 63;
    unsigned long long ex = 0;
    double ob = 0.0;
    for (unsigned long long e = (unsigned long long)blockIdx.x * kWG + threadIdx.x; e < E;
         e += (unsigned long long)gridDim.x * kWG) {
        const EdgeRec rec = A.edges[e];
        const ProbDev pd = A.probs[rec.prob];
        const GramProb gp = P.gp[rec.prob];
        const int gi = pd.var_off + rec.i, gj = pd.var_off + rec.j;
        double stat;
        int64_t df;
        pair_stat(P, gp, P.var_oh[gi], P.var_oh[gj], A.cards[gi], A.cards[gj], pd.m, A.tile.stat,
                  A.tile.df_rule != 0, stat, df);
        if (chi2_tail_lane(df, stat) > pd.alpha) A.min_accept[e] = 0ull;  // the depth's only test accepted
        ++ex;
        ob += 2.0 * (double)pd.m;
        if (A.per_prob) A.ecnt[2 * e] = 1u;
    }
    ex = wave_sum(ex);
    ob = wave_sum(ob);
    if (lane == 0) {
        if (ex) atomicAdd(&c->stats[0].executed, ex);
        if (ob > 0.0) atomicAdd(&c->stats[0].operand_bytes, ob);
        atomicMax(&c->stats[0].t_end, (unsigned long long)wall_clock64());
    }
}

// Every pair i < j of one dataset (all-pairs entry point): pair index
// i n - i (i + 1) / 2 + j - i - 1.
__global__ __launch_bounds__(kWG) void k_ci_pairs(PairArgs P, const uint8_t *cards, int32_t n, double alpha,
                                                  int stat_kind, int df_rule, double *stat_out, int64_t *df_out,
                                                  double *p_out, int32_t *flags_out) {
    const GramProb gp = P.gp[0];
    const int64_t npairs = (int64_t)n * (n - 1) / 2;
    for (int64_t q = (int64_t)blockIdx.x * kWG + threadIdx.x; q < npairs; q += (int64_t)gridDim.x * kWG) {
        // row i: the largest i with i n - i (i + 1) / 2 <= q
        int lo = 0, hi = n - 2;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if ((int64_t)mid * n - (int64_t)mid * (mid + 1) / 2 <= q) lo = mid;
            else hi = mid - 1;
        }
        const int i = lo;
        const int j = (int)(q - ((int64_t)i * n - (int64_t)i * (i + 1) / 2)) + i + 1;
        double stat;
        int64_t df;
        pair_stat(P, gp, P.var_oh[i], P.var_oh[j], cards[i], cards[j], gp.m, stat_kind, df_rule != 0, stat, df);
        const double p = chi2_tail_lane(df, stat);
        if (stat_out) stat_out[q] = stat;
        if (df_out) df_out[q] = df;
        if (p_out) p_out[q] = p;
        if (flags_out) flags_out[q] = p > alpha ? 1 : 0;
    }
}

static int gram_occupancy(int T) {
    int nb = 0;
    const hipError_t e = T == 128 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_gram<128>, kGramWG, 0)
                                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_gram<64>, kGramWG, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

int gram_max_wg_per_cu(int T) { return gram_occupancy(T); }

// The Gram tiles of every problem (and their sum over chunks).
static void launch_gram(const PairArgs &p, Ctl *c, hipStream_t s) {
    const dim3 grid(p.gram_grid);
    if (p.T == 128) hipLaunchKernelGGL(k_gram<128>, grid, dim3(kGramWG), 0, s, p, c);
    else hipLaunchKernelGGL(k_gram<64>, grid, dim3(kGramWG), 0, s, p, c);
    if (p.gram != p.part) {
        const int64_t words = p.tiles * p.T * p.T / 4;
        const int rg = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (words + kWG - 1) / kWG));
        hipLaunchKernelGGL(k_gram_reduce, dim3(rg), dim3(kWG), 0, s, p);
    }
}

hipError_t launch_depth0_pairs(const DepthArgs &a, hipStream_t s) {
    launch_gram(a.pairs, a.ctl, s);
    hipLaunchKernelGGL(k_depth0_pairs, dim3(a.edge_grid), dim3(kWG), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ci_pairs(const PairArgs &p, const uint8_t *cards, int32_t n, double alpha, int stat,
                           int df_rule, double *stat_out, int64_t *df_out, double *p_out, int32_t *flags_out,
                           hipStream_t s) {
    launch_gram(p, nullptr, s);
    const int64_t npairs = (int64_t)n * (n - 1) / 2;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(2048, (npairs + kWG - 1) / kWG));
    hipLaunchKernelGGL(k_ci_pairs, dim3(grid), dim3(kWG), 0, s, p, cards, n, alpha, stat, df_rule, stat_out,
                       df_out, p_out, flags_out);
    return hipGetLastError();
}

}  // namespace bns
