// gfx950 kernels of the batched G^2 CI-test engine and of the per-depth
// PC-stable pipeline (Algorithm 1; grouping, lexicographic conditioning sets
// and depth-0 handling of Sections IV-B and IV-C).
#include <hip/hip_ext.h>

#include <algorithm>

#include "device_ci.h"
#include "kernels.h"

namespace bns {

// ---------------------------------------------------------------------------
// Helpers
// ---------------------------------------------------------------------------
__device__ inline uint64_t binom_at(const uint64_t *B, int rows, int64_t n, int k) {
    if (n < 0 || k < 0 || k > n) return 0;
    if (n >= rows || k >= kBinomK) return ~0ull >> 2;
    return B[n * kBinomK + k];
}

__device__ inline uint64_t lanes_below_mask() {
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Position of rank rr among the size-d subsets of {0..p-1} in lexicographic
// order (one thread, sequential): writes c[0..d).
// A view of the binomial table: C(n, k) at tab[n * stride + k] for n < rows
// (the full table in device memory, or a slice n < rows, k < stride staged
// in LDS); saturated beyond it.
struct Binom {
    const uint64_t *tab;
    int stride;
    int rows;
    __device__ uint64_t at(int64_t n, int k) const {
        if (n < 0 || k < 0 || k > n) return 0;
        if (n >= rows || k >= stride) return ~0ull >> 2;
        return tab[n * stride + k];
    }
};

// Serial lexicographic unranking (one lane): positions of the rank-rr size-d
// subset of {0..p-1}.
// S(x) = number of subsets (with the current prefix) whose k-th element is < x
//      = C(p - x0, j + 1) - C(p - x, j + 1)   (hockey-stick identity)
// is non-decreasing in x, so the k-th element, the largest x in
// [x0, p - j - 1] with S(x) <= rr, is found by bisection.
__device__ inline void unrank_serial(const Binom &B, int64_t p, int d, uint64_t rr, int32_t *c) {
    int64_t x0 = 0;
    for (int k = 0; k < d; ++k) {
        const int j = d - k - 1;
        const uint64_t base = B.at(p - x0, j + 1);
        int64_t lo = x0, hi = p - j - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (base - B.at(p - mid, j + 1) <= rr) lo = mid;
            else hi = mid - 1;
        }
        c[k] = (int32_t)lo;
        rr -= base - B.at(p - lo, j + 1);
        x0 = lo + 1;
    }
}

__global__ void k_ci_batch(const uint8_t *data, int64_t ld, int64_t m, const uint8_t *cards,
                           const CiTestDev *tests, const int32_t *zpool, int64_t n_tests,
                           double alpha, Tile tile, CiOutDev *out, CiOutSoa soa, uint32_t *tables,
                           const int64_t *table_off);
__global__ void k_plain_count(const uint8_t *data, int64_t ld, int64_t m, const uint8_t *cards,
                              const PlainTest pt, int64_t spb, uint32_t *partials, int64_t T,
                              int lds_words);

// Ticket levels of an edge with n tests: with doubling levels (g = 0) level L
// holds ranks [2^L - 1, 2^(L+1) - 1), so 64 - clz(n) levels; with rounds of g
// ranks, ceil(n / g) levels, at most 64 (the last one takes the rest).
BNS_INLINE int edge_levels(uint64_t n, int g) {
    if (n == 0) return 0;
    if (g <= 0) return 64 - __clzll(n);
    const uint64_t k = (n + (uint64_t)g - 1) / (uint64_t)g;
    return k > 64 ? 64 : (int)k;
}

// ---------------------------------------------------------------------------
// Search initialisation: complete graph, no removals, control block reset.
// ---------------------------------------------------------------------------
constexpr int kSmallRows = 1024;
constexpr int64_t kSmallPairs = 65536;

__host__ __device__ bool small_search(const DepthArgs &a) {
    return a.n_globals <= kSmallRows && a.n_pairs <= kSmallPairs && a.bit_words <= kSmallBitWords;
}

__global__ void k_init_search(DepthArgs A) {
    const int pi = blockIdx.y;
    const ProbDev P = A.probs[pi];
    const int64_t nn = (int64_t)P.n * P.n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / P.n, j = e - i * P.n;
        A.adj[P.adj_off + e] = (i != j) ? 1 : 0;
        A.rdepth[P.adj_off + e] = -1;
    }
    if (small_search(A)) {
        // complete graph as bit rows: bits u < n of row v, except u = v
        const int W = (P.n + 63) / 64;
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < P.n * W; e += gridDim.x * blockDim.x) {
            const int v = e / W, w = e - v * W;
            const int lo = 64 * w, nb = min(64, P.n - lo);
            uint64_t word = (nb >= 64) ? ~0ull : ((1ull << nb) - 1ull);
            if (v >= lo && v < lo + 64) word &= ~(1ull << (v - lo));
            A.adjbits[P.bit_off + e] = word;
        }
    }
    if (A.per_prob && blockIdx.x == 0) {
        for (int i = threadIdx.x; i < kMaxDepths; i += blockDim.x) {
            PStatDev z = {};
            A.pstat[(int64_t)pi * kMaxDepths + i] = z;
        }
    }
    if (pi == 0 && blockIdx.x == 0) {
        Ctl *c = A.ctl;
        if (threadIdx.x == 0) {
            if (A.err_cnt) *A.err_cnt = 0ull;
            c->depth = 0;
            c->done = 0;
            c->error = 0;
            c->n_edges = 0;
            c->total_tickets = 0;
            c->pool_used = 0;
            c->apply_done = 0;
            c->gram_depth = -1;
        }
        for (int i = threadIdx.x; i < kMaxDepths; i += blockDim.x) {
            DepthStatDev z = {};
            c->stats[i] = z;
        }
    }
}

// ---------------------------------------------------------------------------
// Depth preparation
// ---------------------------------------------------------------------------

// One wave per variable: freeze a(v) (ascending), its size, and the number of
// surviving edges (v, u) with u > v.
BNS_INLINE void snapshot_row(const DepthArgs &A, int g, int &deg_out, int &hi_out) {
    const int lane = threadIdx.x & 63;
    const ProbDev &P = A.probs[A.var2prob[g]];
    const int v = g - P.var_off, n = P.n;
    const uint8_t *row = A.adj + P.adj_off + (int64_t)v * n;
    int32_t *nb = A.nbr + P.adj_off + (int64_t)v * n;
    int32_t *ip = A.ipos + P.adj_off + (int64_t)v * n;
    const uint64_t lt = lanes_below_mask();
    int cnt = 0, hi = 0;
    for (int u0 = 0; u0 < n; u0 += 64) {
        const int u = u0 + lane;
        const bool a = (u < n) && row[u];
        const uint64_t mask = __ballot(a);
        if (a) {
            const int pos = cnt + __popcll(mask & lt);
            nb[pos] = u;
            ip[u] = pos;
        }
        cnt += __popcll(mask);
        hi += __popcll(__ballot(a && u > v));
    }
    deg_out = cnt;
    hi_out = hi;
}

__global__ __launch_bounds__(kWG) void k_snapshot(DepthArgs A) {
    if (A.ctl->done) return;
    const int g = blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (g < A.n_globals) {
        int dg, hi;
        snapshot_row(A, g, dg, hi);
        if ((threadIdx.x & 63) == 0) {
            A.deg[g] = dg;
            A.rowcnt[g] = hi;
        }
    }
}

// Single workgroup: exclusive scan of the per-variable edge counts, reset of
// the per-depth counters.
__global__ __launch_bounds__(kWG) void k_scan_rows(DepthArgs A) {
    Ctl *c = A.ctl;
    if (c->done) return;
    __shared__ int64_t part[kWG];
    const int G = A.n_globals;
    const int seg = (G + kWG - 1) / kWG;
    const int b = threadIdx.x * seg, e = min(G, b + seg);
    __shared__ int mdeg[kWG];
    int64_t s = 0;
    int md = 0;
    for (int i = b; i < e; ++i) {
        s += A.rowcnt[i];
        md = max(md, A.deg[i]);
    }
    part[threadIdx.x] = s;
    mdeg[threadIdx.x] = md;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int i = 0; i < kWG; ++i) {
            const int64_t v = part[i];
            part[i] = acc;
            acc += v;
        }
        c->n_edges = (unsigned long long)acc;
        int m2 = 0;
        for (int i = 0; i < kWG; ++i) m2 = max(m2, mdeg[i]);
        c->maxdeg = m2;
        c->maxn = 0;
        c->total_tickets = 0;
        if (c->depth >= kMaxDepths) c->error = kDevDepthTooLarge;
    }
    for (int i = threadIdx.x; i < kMaxLevels + 2; i += kWG) c->hist[i] = 0;
    __syncthreads();
    int64_t acc = part[threadIdx.x];
    for (int i = b; i < e; ++i) {
        A.rowbase[i] = acc;
        acc += A.rowcnt[i];
    }
}

// One wave per variable v: an edge record for every surviving (v, u > v) with
// its test counts C(|a(v)|-1, d) + C(|a(u)|-1, d) (one test at depth 0).
BNS_INLINE void edges_row(const DepthArgs &A, Ctl *c, int g, unsigned int *hist) {
    const int lane = threadIdx.x & 63;
    const int pi = A.var2prob[g];
    const ProbDev &P = A.probs[pi];
    const int v = g - P.var_off, n = P.n;
    const int d = c->depth;
    const bool depth_ok = (P.max_depth < 0 || d <= P.max_depth);
    const uint8_t *row = A.adj + P.adj_off + (int64_t)v * n;
    const int dv = A.deg[g];
    const int64_t base = A.rowbase[g];
    const uint64_t lt = lanes_below_mask();
    int cnt = 0, hi = 0;
    unsigned long long tk_sum = 0;  // this lane's tests (per-problem counters)
    for (int u0 = 0; u0 < n; u0 += 64) {
        const int u = u0 + lane;
        const bool a = (u < n) && row[u];
        const uint64_t mask = __ballot(a);
        const bool take = a && u > v;
        const uint64_t mhi = __ballot(take);
        if (take) {
            EdgeRec e;
            e.prob = pi;
            e.i = v;
            e.j = u;
            e.posj = cnt + __popcll(mask & lt);
            const int du = A.deg[P.var_off + u];
            uint64_t nA = 0, nB = 0;
            if (depth_ok) {
                if (d == 0) {
                    nA = 1;
                } else if (d > kMaxZ) {
                    if (dv - 1 >= d || du - 1 >= d) c->error = kDevDepthTooLarge;
                } else {
                    nA = binom_at(A.binom, A.binom_rows, dv - 1, d);
                    nB = binom_at(A.binom, A.binom_rows, du - 1, d);
                }
            }
            uint64_t ntot = nA + nB;
            if (ntot > (1ull << 40)) {
                c->error = kDevTooManyTests;
                nA = nB = ntot = 0;
            }
            e.nA = nA;
            e.n = ntot;
            e.pA = dv - 1;
            e.pB = du - 1;
            e.posi = 0;
            if (nB > 0) e.posi = A.ipos[P.adj_off + (int64_t)u * n + v];  // v in a(u)
            e.levels = edge_levels(ntot, A.round_width);
            atomicAdd(&hist[e.levels], 1u);
            if (A.round_width > 0 && ntot) atomicMax(&c->maxn, (unsigned long long)ntot);
            A.edges_tmp[base + hi + __popcll(mhi & lt)] = e;
            tk_sum += ntot;
        }
        cnt += __popcll(mask);
        hi += __popcll(mhi);
    }
    if (A.per_prob && d < kMaxDepths) {
        tk_sum = wave_sum(tk_sum);
        if (lane == 0) {
            PStatDev &ps = A.pstat[(int64_t)pi * kMaxDepths + d];
            atomicAdd(&ps.edges, (unsigned long long)hi);
            if (tk_sum) atomicAdd(&ps.tickets, tk_sum);
        }
    }
}

__global__ __launch_bounds__(kWG) void k_edges(DepthArgs A) {
    __shared__ unsigned int hist[kMaxLevels + 2];
    Ctl *c = A.ctl;
    const bool live = !c->done;
    for (int i = threadIdx.x; i < kMaxLevels + 2; i += kWG) hist[i] = 0;
    __syncthreads();
    const int g = blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (live && g < A.n_globals && A.rowcnt[g] > 0) edges_row(A, c, g, hist);
    __syncthreads();
    for (int i = threadIdx.x; i < kMaxLevels + 2; i += kWG)
        if (hist[i]) atomicAdd(&c->hist[i], hist[i]);
}

// One wave: ticket levels.  Edges are ordered by their number of levels,
// descending, so the edges with a test of rank r form a prefix; level L holds
// ranks [2^L - 1, 2^(L+1) - 1) of the first level_cnt[L] edges, rank-major.
// Tickets per test wave from which one test per wave beats one per workgroup
// (twice as many from depth kWaveModeDeepDepth on: bigger tables cost a wave
// more passes over its quarter of the LDS and a longer epilogue).
constexpr unsigned long long kWaveModeRounds = 6;
constexpr int kWaveModeDeepDepth = 3;
// Below it, one test per wave also wins at depths up to kWaveModeSmallDepth
// when every wave gets at most one ticket but a workgroup would take two or
// more rounds: the longer single-wave test costs less than the extra rounds
// of per-test latency, and tables of so few columns fit a wave's LDS share.
constexpr int kWaveModeSmallDepth = 2;

BNS_INLINE void levels_wave(const DepthArgs &A, Ctl *c, const unsigned int *hist, int d, int maxdeg,
                            unsigned long long maxn, unsigned int *cursor_lds = nullptr,
                            int *done_lds = nullptr) {
    const int lane = threadIdx.x & 63;
    // binomial slice of the depth for the test kernel, work-unit counters
    const int brows = maxdeg + 1;
    const bool staged = d + 1 <= kBinomK && brows <= A.binom_rows && brows * (d + 1) <= kBinomLds;
    if (staged)
        for (int i = lane; i < brows * (d + 1); i += 64) {
            const int n = i / (d + 1), k = i - n * (d + 1);
            c->bslice[i] = k == 0 ? 1ull : A.binom[n * kBinomK + k];
        }
    if (lane < kGrabParts) c->grab_ctr[lane * kGrabStride] = 0ull;
    // cursor[lv] = number of edges with more than lv levels (bucket start in
    // the descending order); lanes hold lv = lane and lv = 64, 65 go to lane 0.
    const unsigned int h = hist[lane];
    unsigned int suf = h;  // inclusive suffix sum over lanes >= lane
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned int o = __shfl_down(suf, off, 64);
        if (lane + off < 64) suf += o;
    }
    const unsigned int hi = hist[kMaxLevels] + hist[kMaxLevels + 1];
    const unsigned int start = suf - h + hi;  // edges with levels > lane
    c->cursor[lane] = start;
    if (lane == 0) {
        c->cursor[kMaxLevels + 1] = 0;
        c->cursor[kMaxLevels] = hist[kMaxLevels + 1];
    }
    if (cursor_lds) {
        cursor_lds[lane] = start;
        if (lane == 0) {
            cursor_lds[kMaxLevels + 1] = 0;
            cursor_lds[kMaxLevels] = hist[kMaxLevels + 1];
        }
    }
    // level L (= lane): cnt = edges with levels > L, tickets cnt * width(L),
    // width 2^L (doubling) or g (the last of 64 rounds: up to the most tests
    // of an edge)
    const unsigned long long cnt = start;
    const int g = A.round_width;
    // Depth 1 in (edge, level) units: one unit per edge and level, its ranks
    // counted together (doubling levels only; not in verification mode)
    const bool xy = A.xy_policy == 1 && d == 1 && g == 0 && !A.edge_form && A.err_val == nullptr;
    unsigned long long width = 1ull << (lane < 62 ? lane : 62);
    if (g > 0) width = lane < 63 ? (unsigned long long)g
                                 : (maxn > 63ull * g ? maxn - 63ull * g : (unsigned long long)g);
    if (xy) width = 1ull;
    int bad = 0;
    unsigned long long tk = 0;
    if (cnt) {
        if ((g <= 0 && lane >= 60) || cnt > (1ull << 61) / width) bad = 1;
        else tk = cnt * width;
    }
    unsigned long long pre = tk;  // inclusive prefix over lanes <= lane
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long o = __shfl_up(pre, off, 64);
        if (lane >= off) pre += o;
    }
    c->level_base[lane] = pre - tk;
    c->level_cnt[lane] = cnt;
    const unsigned long long total = __shfl(pre, 63, 64);
    const bool any_bad = __ballot(bad) != 0ull;
    if (lane == 0) {
        c->level_base[kMaxLevels] = total;
        c->level_cnt[kMaxLevels] = 0;
        if (any_bad) c->error = kDevTooManyTests;
        c->total_tickets = any_bad ? 0ull : total;
        c->bstride = staged ? d + 1 : 0;
        c->brows = staged ? brows : 0;
        // Group per test: a wave (no workgroup barriers), or a workgroup
        // (4x the LDS and lanes per test: shorter tests, less speculation).
        // Automatic: a workgroup per test unless there are tickets for
        // several rounds of all waves (more at deep depths), or, at shallow
        // depths, for a quarter to one round of them.
        // Per-depth overrides (depths below 32) come first.
        const unsigned long long tw = (unsigned long long)max(A.test_waves, 1);
        const uint32_t dbit = d < 32 ? 1u << d : 0u;
        const int mode = (A.block_depths & dbit) ? 1
                       : (A.wave_depths & dbit)  ? 0
                       : xy                      ? 1  // (edge, level) units: a wave's LDS share holds few tables
                       : (A.mode_policy == 2)    ? 1
                       : (A.mode_policy == 1)    ? 0
                       : (total >= kWaveModeRounds * tw * (d >= kWaveModeDeepDepth ? 2ull : 1ull)) ? 0
                       : (d <= kWaveModeSmallDepth && 4ull * total >= tw && total <= tw) ? 0
                       : 1;
        const unsigned long long groups = mode ? max(tw / kWaves, 1ull) : tw;
        // Fewer tickets than half the groups: cut each test's samples into
        // chunks of at least split_min samples, counted by different groups
        // and merged in device memory (about units_per_group units per group).
        // With more tickets the merges cost more than the idle groups.
        unsigned long long C = 1, cap = 0;
        long long Lc = A.m_max;
        if (!xy && A.split_min > 0 && total > 0 && total <= (unsigned long long)A.split_tickets) {
            const unsigned long long want =
                (unsigned long long)max(A.units_per_group, 1) * groups / total;
            const unsigned long long by_len = (unsigned long long)(A.m_max / A.split_min);
            const unsigned long long cc = min(min(want, by_len), 65536ull);
            // whole 128-byte lines per ticket: no two tickets' tables share a line
            cap = ((unsigned long long)A.split_words / total) & ~31ull;
            if (cc >= 2 && cap >= 64) {
                const long long per = (A.m_max + (long long)cc - 1) / (long long)cc;
                Lc = (per + 1023) & ~1023ll;
                C = (unsigned long long)((A.m_max + Lc - 1) / Lc);
            }
        }
        if (C < 2) {
            C = 1;
            Lc = A.m_max;
            cap = 0;
        }
        c->mode = mode;
        c->xy = xy ? 1 : 0;
        c->chunks = (int)C;
        c->chunk_len = Lc;
        c->split_cap = cap;
        c->total_units = any_bad ? 0ull : total * C;
        // Grabs of several units amortise the decode latency when there is
        // work for many rounds; a group holds its batch, so larger batches
        // also run more tests before earlier ranks of their edges finish
        // (speculation) and leave more work with one group at the end of
        // the depth: one unit per grab per eight rounds of all groups for
        // workgroups, per 32 rounds for waves (a wave's test takes four times
        // as long, and a batch of tests of very different lengths, as in a
        // batch of datasets, ends late).
        const unsigned long long per = total * C / ((mode ? 8ull : 32ull) * groups);
        c->batch = A.grab_fixed > 0 ? A.grab_fixed
                                    : (int)max(1ull, min(per, (unsigned long long)kSlotsPerWave));
        if (done_lds) *done_lds = (total == 0 || any_bad) ? 1 : 0;
        if (total == 0 || any_bad) {
            c->done = 1;
        } else if (d < kMaxDepths) {
            c->stats[d].edges = c->n_edges;
            c->stats[d].tickets = total;
            c->stats[d].mode = mode;
            c->stats[d].chunks = (int32_t)C;
            c->stats[d].chunk_len = Lc;
        }
    }
}

__global__ void k_levels(DepthArgs A) {
    Ctl *c = A.ctl;
    if (c->done) return;
    levels_wave(A, c, c->hist, c->depth, c->maxdeg, c->maxn);
}

// Scatter into level order and reset the per-edge first-accept ranks.  The
// bucket cursors are bumped once per distinct level value per wave.
BNS_INLINE void scatter_edges(const DepthArgs &A, Ctl *c, unsigned long long first,
                              unsigned long long stride) {
    const unsigned long long E = c->n_edges;
    const int lane = threadIdx.x & 63;
    const uint64_t lt = lanes_below_mask();
    for (unsigned long long base = first; base < E; base += stride) {
        const unsigned long long e = base + lane;
        const bool valid = e < E;
        EdgeRec r;
        int lv = -1;
        if (valid) {
            r = A.edges_tmp[e];
            lv = r.levels;
        }
        uint64_t todo = __ballot(valid);
        unsigned int pos = 0;
        while (todo) {
            const int leader = __ffsll((long long)todo) - 1;
            const int L = __shfl(lv, leader, 64);
            const uint64_t same = __ballot(valid && lv == L);
            unsigned int b = 0;
            if (lane == leader) b = atomicAdd(&c->cursor[L], (unsigned int)__popcll(same));
            b = __shfl(b, leader, 64);
            if (valid && lv == L) pos = b + (unsigned int)__popcll(same & lt);
            todo &= ~same;
        }
        if (valid) {
            A.edges[pos] = r;
            A.min_accept[pos] = ~0ull;
            if (A.per_prob) {
                A.ecnt[2 * (uint64_t)pos] = 0u;
                A.ecnt[2 * (uint64_t)pos + 1] = 0u;
            }
        }
    }
}

__global__ __launch_bounds__(kWG) void k_scatter(DepthArgs A) {
    Ctl *c = A.ctl;
    if (c->done) return;
    scatter_edges(A, c, (unsigned long long)blockIdx.x * kWG + (threadIdx.x & ~63u),
                  (unsigned long long)gridDim.x * kWG);
}

// ---------------------------------------------------------------------------
// Small searches (at most kSmallRows variables and kSmallPairs pairs in all):
// one workgroup prepares a depth (k_prepare_small, first depth) or removes
// the accepted edges of a depth and prepares the next (k_apply_small), with
// the per-variable state in LDS.  Edge records go straight to their slot in
// the level order (a first pass over the rows counts the levels, a second
// writes the records).
// ---------------------------------------------------------------------------
constexpr int kSmallThreads = 1024;
constexpr int kSmallWaves = kSmallThreads / 64;

constexpr int kSmallProbs = 8;      // problem records staged in LDS
constexpr int kApplyBinom = 1024;   // binomials C(n, k <= d) staged for the removal records

struct SmallSh {
    uint64_t bits[kSmallBitWords];  // adjacency bit rows of all problems
    uint64_t btab[kApplyBinom];
    ProbDev probs[kSmallProbs];
    uint64_t bcol[kSmallRows];  // C(x, d) for x <= max degree
    int deg[kSmallRows];
    int rowcnt[kSmallRows];
    unsigned int hist[kMaxLevels + 2];
    unsigned int cursor[kMaxLevels + 2];
    unsigned long long red[2][kSmallWaves];
    int wmax[kSmallWaves];
    int done;
    // control-block header, read once
    int h_done, h_depth, h_maxdeg, h_bstride, h_brows;
    unsigned long long h_edges;
    unsigned long long pool_ctr;  // removal-record words used (the removal kernel's own counter)
    unsigned long long maxn;      // most tests of one edge at the depth being prepared
};

// Tests of edge (v, u) at depth d from the frozen degrees (0 when the depth
// is beyond the problem's max_depth); sets an error for impossible counts.
BNS_INLINE void small_counts(Ctl *c, const SmallSh &sh, bool depth_ok, int d, int dv, int du,
                             uint64_t &nA, uint64_t &nB) {
    nA = nB = 0;
    if (!depth_ok) return;
    if (d == 0) {
        nA = 1;
    } else if (d > kMaxZ) {
        if (dv - 1 >= d || du - 1 >= d) c->error = kDevDepthTooLarge;
    } else {
        nA = (dv >= 1) ? sh.bcol[dv - 1] : 0;
        nB = (du >= 1) ? sh.bcol[du - 1] : 0;
    }
    if (nA + nB > (1ull << 40)) {
        c->error = kDevTooManyTests;
        nA = nB = 0;
    }
}

// Problem of global variable g: from the LDS copies when there are few problems.
BNS_INLINE int small_prob_index(const DepthArgs &A, const SmallSh &sh, int g) {
    if (A.n_probs > kSmallProbs) return A.var2prob[g];
    int pi = 0;
    for (int k = 1; k < A.n_probs; ++k)
        if (sh.probs[k].var_off <= g) pi = k;
    return pi;
}
BNS_INLINE const ProbDev &small_prob(const DepthArgs &A, const SmallSh &sh, int pi) {
    return A.n_probs > kSmallProbs ? A.probs[pi] : sh.probs[pi];
}

// Stages the bit rows and problem records of a small search in LDS.
BNS_INLINE void small_load(const DepthArgs &A, SmallSh &sh) {
    for (int i = threadIdx.x; i < A.bit_words; i += kSmallThreads) sh.bits[i] = A.adjbits[i];
    if (A.n_probs <= kSmallProbs && threadIdx.x < (unsigned)A.n_probs) sh.probs[threadIdx.x] = A.probs[threadIdx.x];
}

// Bit u of row v of a problem's adjacency bit rows (W words per row).
BNS_INLINE bool bit_at(const uint64_t *rows, int W, int v, int u) {
    return (rows[v * W + (u >> 6)] >> (u & 63)) & 1ull;
}

// Set bits of row v below u: the position of u in the ascending list of v.
BNS_INLINE int bits_below(const uint64_t *rows, int W, int v, int u) {
    const uint64_t *r = rows + v * W;
    int c = 0;
    for (int w = 0; w < (u >> 6); ++w) c += __popcll(r[w]);
    return c + __popcll(r[u >> 6] & ((1ull << (u & 63)) - 1ull));
}

// Item i of the bit rows (one 64-bit word of one row): problem, row, word.
struct BitItem {
    int pi, v, w, W;
};
BNS_INLINE BitItem bit_item(const DepthArgs &A, const SmallSh &sh, int i) {
    int pi = 0;
    if (A.n_probs <= kSmallProbs) {
        for (int k = 1; k < A.n_probs; ++k)
            if (sh.probs[k].bit_off <= i) pi = k;
    } else {
        int lo = 0, hi = A.n_probs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (A.probs[mid].bit_off <= i) lo = mid;
            else hi = mid - 1;
        }
        pi = lo;
    }
    const ProbDev &P = small_prob(A, sh, pi);
    const int W = (P.n + 63) >> 6;
    const int r = i - P.bit_off;
    const int v = r / W;
    return BitItem{pi, v, r - v * W, W};
}

// Bits of word w (bits 64w .. 64w + 63) above index v.
BNS_INLINE uint64_t bits_above(uint64_t x, int w, int v) {
    const int lo = 64 * w;
    if (v < lo) return x;
    if (v >= lo + 63) return 0ull;
    return x & (~0ull << (v - lo + 1));
}

// Preparation of depth d by one workgroup from the bit rows in LDS.  Work is
// spread one thread per variable (degrees) or per slice of a row word
// (lists, levels, records): each word is cut into L slices of 64 / L bits,
// L a power of two chosen so that the slices about fill the workgroup.
BNS_INLINE void prepare_block(const DepthArgs &A, Ctl *c, int d, SmallSh &sh) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int G = A.n_globals;
    const int NW = (int)A.bit_words;
    int lgL = 0;
    while (lgL < 6 && (NW << (lgL + 1)) <= kSmallThreads) ++lgL;
    const int NS = NW << lgL;            // slices
    const int sbits = 64 >> lgL;         // bits per slice
    const uint64_t smask = (sbits == 64) ? ~0ull : ((1ull << sbits) - 1ull);
    for (int i = threadIdx.x; i < kMaxLevels + 2; i += kSmallThreads) sh.hist[i] = 0;
    if (threadIdx.x == 0) sh.maxn = 0;
    // degrees and higher-neighbour counts, one thread per variable
    for (int g = threadIdx.x; g < G; g += kSmallThreads) {
        const ProbDev &P = small_prob(A, sh, small_prob_index(A, sh, g));
        const int v = g - P.var_off, W = (P.n + 63) >> 6;
        const uint64_t *row = sh.bits + P.bit_off + v * W;
        int cnt = 0, hi = 0;
        for (int k = 0; k < W; ++k) {
            const uint64_t x = row[k];
            cnt += __popcll(x);
            hi += __popcll(bits_above(x, k, v));
        }
        sh.deg[g] = cnt;
        sh.rowcnt[g] = hi;
    }
    __syncthreads();
    // frozen adjacency lists (ascending), one thread per row word; edge total
    // and largest degree
    for (int i = threadIdx.x; i < NS; i += kSmallThreads) {
        const BitItem it = bit_item(A, sh, i >> lgL);
        const int s0 = (i & ((1 << lgL) - 1)) * sbits;  // first bit of the slice
        const ProbDev &P = small_prob(A, sh, it.pi);
        const uint64_t *row = sh.bits + P.bit_off + it.v * it.W;
        int pos = 0;
        for (int k = 0; k < it.w; ++k) pos += __popcll(row[k]);
        const uint64_t word = row[it.w];
        if (s0) pos += __popcll(word & ((1ull << s0) - 1ull));
        int32_t *nb = A.nbr + P.adj_off + (int64_t)it.v * P.n;
        uint64_t x = word & (smask << s0);
        while (x) {
            nb[pos++] = 64 * it.w + __ffsll((long long)x) - 1;
            x &= x - 1ull;
        }
    }
    {
        int64_t s = 0;
        int md = 0;
        for (int g = threadIdx.x; g < G; g += kSmallThreads) {
            s += sh.rowcnt[g];
            md = max(md, sh.deg[g]);
        }
        s = wave_sum(s);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) md = max(md, __shfl_xor(md, off, 64));
        if (lane == 0) {
            sh.red[0][w] = (unsigned long long)s;
            sh.wmax[w] = md;
        }
    }
    __syncthreads();
    int maxdeg = 0;
    unsigned long long E = 0;
    for (int i = 0; i < kSmallWaves; ++i) {
        E += sh.red[0][i];
        maxdeg = max(maxdeg, sh.wmax[i]);
    }
    for (int x = threadIdx.x; x <= maxdeg && d <= kMaxZ; x += kSmallThreads)
        sh.bcol[x] = d == 0 ? 1ull : binom_at(A.binom, A.binom_rows, x, d);
    if (threadIdx.x == 0) {
        c->n_edges = E;
        c->maxdeg = maxdeg;
        c->total_tickets = 0;
        if (d >= kMaxDepths) c->error = kDevDepthTooLarge;
    }
    __syncthreads();
    // pass 1: level histogram, one thread per row word
    for (int i = threadIdx.x; i < NS; i += kSmallThreads) {
        const BitItem it = bit_item(A, sh, i >> lgL);
        const int s0 = (i & ((1 << lgL) - 1)) * sbits;
        const ProbDev &P = small_prob(A, sh, it.pi);
        const bool depth_ok = (P.max_depth < 0 || d <= P.max_depth);
        const int dv = sh.deg[P.var_off + it.v];
        uint64_t x = bits_above(sh.bits[P.bit_off + it.v * it.W + it.w], it.w, it.v) & (smask << s0);
        while (x) {
            const int u = 64 * it.w + __ffsll((long long)x) - 1;
            x &= x - 1ull;
            uint64_t nA, nB;
            small_counts(c, sh, depth_ok, d, dv, sh.deg[P.var_off + u], nA, nB);
            const uint64_t nt = nA + nB;
            atomicAdd(&sh.hist[edge_levels(nt, A.round_width)], 1u);
            if (A.round_width > 0 && nt) atomicMax(&sh.maxn, (unsigned long long)nt);
        }
    }
    __syncthreads();
    if (w == 0) levels_wave(A, c, sh.hist, d, maxdeg, sh.maxn, sh.cursor, &sh.done);
    __syncthreads();
    if (sh.done) return;
    // pass 2: edge records in level order, one thread per row word
    for (int i = threadIdx.x; i < NS; i += kSmallThreads) {
        unsigned long long n_e = 0, n_tk = 0;  // per-problem counters of this slice
        const BitItem it = bit_item(A, sh, i >> lgL);
        const int s0 = (i & ((1 << lgL) - 1)) * sbits;
        const ProbDev &P = small_prob(A, sh, it.pi);
        const bool depth_ok = (P.max_depth < 0 || d <= P.max_depth);
        const uint64_t *rows = sh.bits + P.bit_off;
        const uint64_t *row = rows + it.v * it.W;
        const int dv = sh.deg[P.var_off + it.v];
        int pos = 0;  // position of the next neighbour in the list of v
        for (int k = 0; k < it.w; ++k) pos += __popcll(row[k]);
        const uint64_t word = row[it.w];
        if (s0) pos += __popcll(word & ((1ull << s0) - 1ull));  // neighbours before the slice
        const uint64_t sl = word & (smask << s0);
        const uint64_t above = bits_above(sl, it.w, it.v);
        pos += __popcll(sl & ~above);  // neighbours of the slice below v come first
        uint64_t x = above;
        while (x) {
            const int u = 64 * it.w + __ffsll((long long)x) - 1;
            x &= x - 1ull;
            const int du = sh.deg[P.var_off + u];
            uint64_t nA, nB;
            small_counts(c, sh, depth_ok, d, dv, du, nA, nB);
            EdgeRec e;
            e.prob = it.pi;
            e.i = it.v;
            e.j = u;
            e.posj = pos++;
            e.posi = (nB > 0) ? bits_below(rows, it.W, u, it.v) : 0;
            e.pA = dv - 1;
            e.pB = du - 1;
            e.nA = nA;
            e.n = nA + nB;
            e.levels = edge_levels(e.n, A.round_width);
            const unsigned int slot = atomicAdd(&sh.cursor[e.levels], 1u);
            A.edges[slot] = e;
            A.min_accept[slot] = ~0ull;
            if (A.per_prob) {
                A.ecnt[2 * (uint64_t)slot] = 0u;
                A.ecnt[2 * (uint64_t)slot + 1] = 0u;
                ++n_e;
                n_tk += e.n;
            }
        }
        if (n_e && d < kMaxDepths) {
            PStatDev &ps = A.pstat[(int64_t)it.pi * kMaxDepths + d];
            atomicAdd(&ps.edges, n_e);
            if (n_tk) atomicAdd(&ps.tickets, n_tk);
        }
    }
}

__global__ __launch_bounds__(kSmallThreads) void k_prepare_small(DepthArgs A) {
    __shared__ SmallSh sh;
    Ctl *c = A.ctl;
    if (threadIdx.x == 0) {
        sh.h_done = c->done;
        sh.h_depth = c->depth;
    }
    small_load(A, sh);
    __syncthreads();
    if (sh.h_done) return;
    prepare_block(A, c, sh.h_depth, sh);
}

// ---------------------------------------------------------------------------
// Persistent per-depth test kernel.
//
// A ticket names (edge, rank r); the conditioning set is unranked on the fly
// from r (Section IV-C) over the frozen adjacency list of side A (lower id)
// for r < nA, else side B.  A test
// whose rank exceeds the smallest accepting rank already found for its edge
// is skipped; since every rank below the final smallest accepting rank is
// always run, the edge's first accepting set in the sequential order is found
// exactly, whatever the interleaving.
//
// Tickets are taken `batch` at a time and decoded lane-parallel into LDS
// descriptors (one lane per ticket), so the dependent loads of a ticket
// (edge record, neighbour lists, cardinalities) cost one latency chain per
// batch.  Mode 0 runs one test per wave in a quarter of the workgroup's LDS;
// mode 1 runs one test per workgroup in all of it.
// ---------------------------------------------------------------------------
struct Desc {
    const uint8_t *data;
    int64_t ld;
    int64_t m;
    double alpha;
    unsigned long long r;
    int64_t e;
    unsigned long long tk;  // ticket
    int32_t chunk;          // sample chunk of the ticket (split depths)
    int32_t prob;
    int32_t valid;
    int32_t ncols;
    uint32_t xyk;            // (edge, level) units: ranks r .. r + xyk - 1 of the edge
    uint16_t var[kMaxCols];  // variable ids (n <= 65535)
    uint8_t card[kMaxCols];
};

constexpr int kProbsLds = 8;     // problem records staged in LDS (searches of few problems)
constexpr int kCardsLds = 2048;  // cardinalities staged in LDS (searches of few variables)

BNS_INLINE uint64_t bnm(const uint64_t *tab, int stride, int rows, int64_t n, int k) {
    if (n < 0 || k < 0 || k > n) return 0;
    if (n >= rows) return ~0ull >> 2;
    return tab[n * stride + k];
}

// Lexicographic unranking by one lane: position c_k of the rank-rr size-d
// subset of {0..p-1}; S(x) = C(p - x0, j + 1) - C(p - x, j + 1) counts the
// subsets with the current prefix whose next element is below x
// (hockey-stick identity).  Writes the positions to out[0..d).
BNS_INLINE void unrank_lane(const uint64_t *tab, int stride, int rows, int64_t p, int d,
                            uint64_t rr, uint16_t *out) {
    int64_t x0 = 0;
    for (int k = 0; k < d; ++k) {
        const int j = d - k - 1;
        const uint64_t base = bnm(tab, stride, rows, p - x0, j + 1);
        // largest x in [x0, p - j - 1] with S(x) <= rr, by bisection
        int64_t lo = x0, hi = p - j - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (base - bnm(tab, stride, rows, p - mid, j + 1) <= rr) lo = mid;
            else hi = mid - 1;
        }
        out[k] = (uint16_t)lo;
        rr -= base - bnm(tab, stride, rows, p - lo, j + 1);
        x0 = lo + 1;
    }
}

BNS_INLINE void decode_edge_rank(const DepthArgs &A, int64_t e, unsigned long long r, const EdgeRec &rec, int d,
                                 const uint64_t *btab, int bstride, int brows, const ProbDev *probs_lds,
                                 const uint8_t *cards_lds, Desc &q);

BNS_INLINE void decode_ticket(const DepthArgs &A, const unsigned long long *lvl_base,
                              const unsigned long long *lvl_cnt, int nlev, unsigned long long tk,
                              int d, const uint64_t *btab, int bstride, int brows, bool skip_ok,
                              const ProbDev *probs_lds, const uint8_t *cards_lds, Desc &q) {
    int lo = 0, hi = nlev - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (lvl_base[mid] <= tk) lo = mid;
        else hi = mid - 1;
    }
    const int L = lo;
    const unsigned long long off = tk - lvl_base[L];
    const unsigned long long cnt = lvl_cnt[L];
    // (a 32-bit division when both fit: much shorter than the 64-bit one)
    const unsigned long long jj = ((off | cnt) >> 32) ? off / cnt
                                                      : (unsigned long long)((uint32_t)off / (uint32_t)cnt);
    const int64_t e = (int64_t)(off - jj * cnt);
    const unsigned long long r =
        (A.round_width > 0 ? (unsigned long long)L * (unsigned long long)A.round_width : ((1ull << L) - 1ull)) + jj;
    const EdgeRec rec = A.edges[e];
    const unsigned long long ma =
        __hip_atomic_load(&A.min_accept[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    q.valid = (r < rec.n && (!skip_ok || r <= ma)) ? 1 : 0;
    // (edge, level) units (width-1 levels of doubling ranks): the level's ranks
    q.xyk = (uint32_t)min(1ull << (L < 62 ? L : 62), r < rec.n ? rec.n - r : 0ull);
    if (!q.valid) return;
    decode_edge_rank(A, e, r, rec, d, btab, bstride, brows, probs_lds, cards_lds, q);
}

// The test of rank r of edge e (record rec) at depth d: its columns,
// cardinalities and sample range (one lane).
BNS_INLINE void decode_edge_rank(const DepthArgs &A, int64_t e, unsigned long long r, const EdgeRec &rec, int d,
                                 const uint64_t *btab, int bstride, int brows, const ProbDev *probs_lds,
                                 const uint8_t *cards_lds, Desc &q) {
    ProbDev P;
    if (probs_lds) P = probs_lds[rec.prob];
    else P = A.probs[rec.prob];
    q.data = P.data;
    q.ld = P.ld;
    q.m = P.m;
    q.alpha = P.alpha;
    q.r = r;
    q.e = e;
    q.prob = rec.prob;
    q.ncols = d + 2;
    q.var[0] = (uint16_t)rec.i;
    q.var[1] = (uint16_t)rec.j;
    if (d > 0) {
        const bool sideA = r < rec.nA;
        const int owner = sideA ? rec.i : rec.j;
        const int skip = sideA ? rec.posj : rec.posi;
        const int64_t p = sideA ? rec.pA : rec.pB;
        unrank_lane(btab, bstride, brows, p, d, sideA ? r : r - rec.nA, q.var + 2);
        // positions -> variable ids, up to 8 loads in flight at a time
        const int32_t *nbo = A.nbr + P.adj_off + (int64_t)owner * P.n;
        // (unconditional loads at a clamped, always valid position, so that
        // all of them are in flight together)
        for (int k0 = 0; k0 < d; k0 += 8) {
            uint32_t vv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int pos = (k0 + k < d) ? q.var[2 + k0 + k] : 0;
                vv[k] = (uint32_t)nbo[pos + (pos >= skip ? 1 : 0)];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (k0 + k < d) q.var[2 + k0 + k] = (uint16_t)vv[k];
        }
    }
    if (cards_lds) {
        const uint8_t *cards = cards_lds + P.var_off;
        for (int k = 0; k < d + 2; ++k) q.card[k] = cards[q.var[k]];
        return;
    }
    const uint8_t *cards = A.cards + P.var_off;
    for (int k0 = 0; k0 < d + 2; k0 += 8) {
        uint32_t cc[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) cc[k] = cards[(k0 + k < d + 2) ? q.var[k0 + k] : 0];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k0 + k < d + 2) q.card[k0 + k] = (uint8_t)cc[k];
    }
}

// Stages a decoded test into the group's TestSh (all lanes of the group).
BNS_INLINE void stage_test(const Grp &g, const Desc &q, TestSh &t) {
    for (int k = g.rank; k < q.ncols; k += g.size) {
        t.col[k] = q.data + (int64_t)q.var[k] * q.ld;
        t.card[k] = q.card[k];
    }
    if (g.rank == 0) {
        t.ncols = q.ncols;
        t.m = q.m;
        uint32_t mlt = 1;
        for (int k = 0; k < q.ncols; ++k) {
            t.mult[k] = mlt;
            mlt *= q.card[k];
        }
    }
    g.sync();
}

BNS_INLINE unsigned long long bcast_u64(unsigned long long v) {
    const unsigned lo = __shfl((unsigned)(v & 0xffffffffull), 0, 64);
    const unsigned hi = __shfl((unsigned)(v >> 32), 0, 64);
    return ((unsigned long long)hi << 32) | lo;
}

// Cells of the test staged in t (saturates above 2^32).
BNS_INLINE uint64_t table_cells(const TestSh &t) {
    uint64_t T = 1;
    for (int k = 0; k < t.ncols && T <= 0xffffffffull; ++k) T *= t.card[k];
    return T;
}

// ---------------------------------------------------------------------------
// Depth 1 in (edge, level) units: the ranks an edge has in one level of the
// work queue differ only in Z, so they are counted in one pass over the
// samples that loads the X and Y columns once (Section IV-B groups the tests
// of an edge for the same reason) and adds every test's own table; their
// epilogues then run together: one table per wave (replica sums, marginals,
// statistic, df) and one chi-square tail per lane.  A pass holds up to kXY
// tests; a unit with more runs in several passes and stops after the pass
// with the first acceptance.
// ---------------------------------------------------------------------------
constexpr int kXY = 8;
constexpr int kPassCols = 3;  // x, y, z

struct PassTest {
    const uint8_t *col[kPassCols];
    uint32_t mult[kPassCols];
    int32_t ncols;
    uint32_t rx, ry, nz;  // cardinalities of X and Y, strata (prod r_Z)
    int64_t e;            // edge record
    uint64_t r;           // rank
    int64_t m;
    double alpha;
};

// Descriptor of a pass, at an 8-byte boundary of the group's LDS region.
struct PassHdr {
    PassTest t[kXY];
    double g2[kXY];
    double df[kXY];
    uint32_t toff[kXY];   // word offset of test i's replicated counts after the header
    uint32_t roff[kXY];   // word offset of its summed table (= toff when not replicated)
    uint32_t moff[kXY];   // word offset of its marginals: rows, columns, strata
    int32_t flag[kXY];    // FP64 re-check requests
    int32_t first;        // first accepting test of the pass (kXY: none)
    int32_t stop;         // the unit's remaining ranks are not needed (group-wide decision)
};
constexpr uint32_t kPassHdrWords = (uint32_t)((sizeof(PassHdr) + 15) / 16 * 4);

struct XYOut {
    int32_t first_accept;  // offset in the unit of its first accepting test, -1: none
    uint32_t exec, rechecks;
    int32_t err;
};

// Density of the chi-square tail's gamma variate at x = g2 / 2 (slope of the
// tail in x), per lane.
BNS_INLINE double chi2_dens_lane(double df, double g2) {
    const double x = 0.5 * g2, a = 0.5 * df;
    if (!(x > 0.0) || !(a > 0.0)) return 0.0;
    return exp((a - 1.0) * log(x) - x - lgamma(a));
}

BNS_INLINE PassHdr &pass_hdr(uint32_t *region, uint32_t **tabs) {
    uint32_t *hreg = region + ((lds_offset(region) >> 2) & 1u);
    *tabs = hreg + kPassHdrWords;
    return *(PassHdr *)hreg;
}

// The most tests of the pass (and then the most replication) whose tables
// fit wt words with 16-bit byte addresses; cells[i]: test i's cells.
BNS_INLINE void pass_plan(const uint32_t (&cells)[kXY], const uint32_t (&marg)[kXY], int kmax, uint32_t wt,
                          uint32_t tab_lo, int max_rep_log2, int64_t msamp, int S, int *kb_out, int *logR_out) {
    int kb = kmax, logR = max_rep_log2;
    for (;;) {
        uint32_t rep_w = 0, red_w = 0, mar_w = 0, cmax = 0;
#pragma unroll
        for (int i = 0; i < kXY; ++i)
            if (i < kb) {
                rep_w += cells[i] << logR;
                red_w += logR > 0 ? cells[i] : 0u;
                mar_w += marg[i];
                cmax = max(cmax, cells[i]);
            }
        const bool fits = (uint64_t)rep_w + red_w + mar_w <= wt && (uint64_t)tab_lo + 4ull * rep_w <= 65536ull;
        const bool cheap = logR == 0 || ((int64_t)(cmax << logR) * 4 <= msamp + 16 * S);
        if (fits && cheap) break;
        if (logR > 0) --logR;
        else if (--kb == 0) break;
    }
    *kb_out = kb;
    *logR_out = logR;
}

// Layout of a pass (lane 0): replicated tables, then per test its summed
// table (when replicated) and its marginals.
BNS_INLINE void pass_layout(PassHdr &h, const uint32_t (&cells)[kXY], const uint32_t (&marg)[kXY], int kb,
                            int logR) {
    uint32_t off = 0;
    for (int i = 0; i < kb; ++i) {
        h.toff[i] = off;
        off += cells[i] << logR;
    }
    for (int i = 0; i < kb; ++i) {
        h.roff[i] = h.toff[i];
        if (logR > 0) {
            h.roff[i] = off;
            off += cells[i];
        }
        h.moff[i] = off;
        off += marg[i];
    }
    h.first = kXY;
}

// Epilogue of a counted pass: per test (one wave each) replica sums,
// marginals, statistic and df; then per test (lane i of the group) the tail,
// an FP64 re-check near alpha from the resident table, and the decision.
// Returns the acceptance of test g.rank (lanes below kb) and, uniform, the
// number of re-checked tests.
template <bool kGeneral>
BNS_INLINE bool pass_finish(const Grp &g, PassHdr &h, uint32_t *tabs, int kb, int logR, const Tile &tile,
                            int *nflag_out) {
    const int nw = g.block ? kWaves : 1;
    const int wv = g.block ? (int)(threadIdx.x >> 6) : 0;
    const int lane = (int)(threadIdx.x & 63);
    const Grp wg = Grp::wave();
    const int stat = kGeneral ? tile.stat : 0;
    const bool adj = kGeneral && tile.df_rule != 0;
    const bool fp64 = tile.fp64 != 0;
    for (int i = wv; i < kb; i += nw) {
        const uint32_t rx = h.t[i].rx, ry = h.t[i].ry, nz = h.t[i].nz;
        const uint32_t Tc = rx * ry * nz;
        uint32_t *red = tabs + h.roff[i];
        if (logR > 0) {
            reduce_replicas(tabs + h.toff[i], red, Tc, logR, lane, 64);
            wg.sync();
        }
        uint32_t *rows = tabs + h.moff[i], *cols = rows + rx * nz, *strata = cols + ry * nz;
        marginals(wg, red, rows, cols, strata, rx, ry, nz);
        double st;
        if (fp64) st = wave_sum(stat_partial<double>(wg, red, rows, cols, strata, rx, ry, nz, stat));
        else st = (double)wave_sum(stat_partial<float>(wg, red, rows, cols, strata, rx, ry, nz, stat));
        const double dfv = adj ? wave_sum(adj_df_partial(wg, rows, cols, strata, rx, ry, nz))
                               : (double)(rx - 1) * (double)(ry - 1) * (double)nz;
        if (lane == 0) {
            h.g2[i] = stat ? st : 2.0 * st;
            h.df[i] = dfv;
        }
    }
    g.sync();
    bool acc = false;
    if (g.rank < kb) {
        const PassTest &q = h.t[g.rank];
        const double x = h.g2[g.rank], df = h.df[g.rank];
        const double p = chi2_tail_lane((int64_t)df, x);
        int flag = 0;
        if (!fp64 && df > 0.0) {
            const double gap = fabs(p - q.alpha);
            const double cells = (double)q.rx * (double)q.ry * (double)q.nz;
            const double rel = (32.0 + cells / 64.0 + 1.0) * 5.96e-8 + 1e-6;
            const double dp = chi2_dens_lane(df, x) * 0.5 * x * rel;
            if (gap < tile.band || gap < 4.0 * dp) flag = 1;
        }
        h.flag[g.rank] = flag;
        acc = !flag && p > q.alpha;
    }
    g.sync();
    int nflag = 0;
#pragma unroll
    for (int i = 0; i < kXY; ++i)
        if (i < kb) nflag += h.flag[i];
    nflag = uni(nflag);
    if (nflag > 0) {
        for (int i = wv; i < kb; i += nw) {
            if (!h.flag[i]) continue;
            const uint32_t rx = h.t[i].rx, ry = h.t[i].ry, nz = h.t[i].nz;
            const uint32_t *red = tabs + h.roff[i];
            const uint32_t *rows = tabs + h.moff[i], *cols = rows + rx * nz, *strata = cols + ry * nz;
            const double st = wave_sum(stat_partial<double>(wg, red, rows, cols, strata, rx, ry, nz, stat));
            if (lane == 0) h.g2[i] = stat ? st : 2.0 * st;
        }
        g.sync();
        if (g.rank < kb && h.flag[g.rank])
            acc = chi2_tail_lane((int64_t)h.df[g.rank], h.g2[g.rank]) > h.t[g.rank].alpha;
    }
    *nflag_out = nflag;
    return acc;
}

// Counts kb tables of one (edge, level) pass: table t at byte offset bt_t
// (+4 replica) counts cell x + rx y + rx ry z_t; two samples per register
// (as count_packed).
BNS_INLINE void count_xy(const uint8_t *xc, const uint8_t *yc, const PassHdr &h, uint32_t tab_lo, int kb,
                         uint32_t rx, uint32_t rxy, int logR, int64_t m, int rank, int S) {
    const uint32_t rep = (uint32_t)rank & ((1u << logR) - 1u);
    const uint32_t mx4 = __builtin_amdgcn_readfirstlane(1u << (logR + 2));
    const uint32_t my4 = __builtin_amdgcn_readfirstlane(rx << (logR + 2));
    const uint32_t mz4 = __builtin_amdgcn_readfirstlane(rxy << (logR + 2));
    // per test: its table's byte offset (scalar) and Z column (scalar)
    uint32_t bt[kXY];
    const gvec4 *cz[kXY];
#pragma unroll
    for (int t = 0; t < kXY; ++t) {
        bt[t] = __builtin_amdgcn_readfirstlane(tab_lo + 4u * h.toff[t < kb ? t : 0]);
        cz[t] = uniform_col(h.t[t < kb ? t : 0].col[2]);
    }
    const uint32_t rep4 = 4u * rep, rep2 = rep4 | (rep4 << 16);
    const gvec4 *cx = uniform_col(xc), *cy = uniform_col(yc);
    const uint32_t nvec = (uint32_t)(m >> 4);
    for (uint32_t i = (uint32_t)rank; i < nvec; i += (uint32_t)S) {
        const u32x4 vx = cx[i], vy = cy[i];
        u32x4 vz[kXY];
#pragma unroll
        for (int t = 0; t < kXY; ++t)
            if (t < kb) vz[t] = cz[t][i];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t bl = mad24(__builtin_amdgcn_perm(0u, vx[j], 0x0c020c00u), mx4,
                                      mad24(__builtin_amdgcn_perm(0u, vy[j], 0x0c020c00u), my4, 0u));
            const uint32_t bh = mad24(__builtin_amdgcn_perm(0u, vx[j], 0x0c030c01u), mx4,
                                      mad24(__builtin_amdgcn_perm(0u, vy[j], 0x0c030c01u), my4, 0u));
#pragma unroll
            for (int t = 0; t < kXY; ++t) {
                if (t >= kb) break;  // uniform
                const uint32_t b2 = (bt[t] | (bt[t] << 16)) + rep2;
                const uint32_t al = mad24(__builtin_amdgcn_perm(0u, vz[t][j], 0x0c020c00u), mz4, bl + b2);
                const uint32_t ah = mad24(__builtin_amdgcn_perm(0u, vz[t][j], 0x0c030c01u), mz4, bh + b2);
                lds_inc(al & 0xffffu);
                lds_inc(al >> 16);
                lds_inc(ah & 0xffffu);
                lds_inc(ah >> 16);
            }
        }
    }
    // the last m mod 16 samples, one per lane
    const int64_t s = ((int64_t)nvec << 4) + rank;
    if (s < m) {
        const uint32_t bxy = ((uint32_t)xc[s] + rx * (uint32_t)yc[s]) << (logR + 2);
#pragma unroll
        for (int t = 0; t < kXY; ++t) {
            if (t >= kb) break;
            const uint8_t *zcol = (const uint8_t *)cz[t];
            lds_inc(bt[t] + rep4 + bxy + ((rxy * (uint32_t)zcol[s]) << (logR + 2)));
        }
    }
}

// Ranks q.r .. q.r + q.xyk - 1 of edge q.e at depth 1 (all lanes of the group).
template <bool kGeneral>
BNS_INLINE XYOut run_xy_unit(const Grp &g, uint32_t *region, uint32_t W, const Tile &tile, const DepthArgs &A,
                             const Desc &q) {
    XYOut o{-1, 0u, 0u, kDevOk};
    uint32_t *tabs;
    PassHdr &h = pass_hdr(region, &tabs);
    const uint32_t Wt = W > kPassHdrWords + 1u ? W - kPassHdrWords - 1u : 0u;
    const uint32_t rx = uni((uint32_t)q.card[0]), ry = uni((uint32_t)q.card[1]), rxy = rx * ry;
    const int64_t m = uni(q.m);
    const int64_t e = uni(q.e);
    const unsigned long long r0 = uni(q.r);
    const uint32_t k = uni(q.xyk);
    const EdgeRec rec = A.edges[e];
    const ProbDev P = A.probs[uni(q.prob)];
    const uint8_t *xc = uni(q.data + (int64_t)q.var[0] * q.ld);
    const uint8_t *yc = uni(q.data + (int64_t)q.var[1] * q.ld);
    const uint32_t tab_lo = lds_offset(tabs);
    uint32_t b0 = 0;
    while (b0 < k) {
        if (b0 > 0) {
            // a lower rank of the edge has accepted: the rest are not needed.
            // One lane reads the edge's first-accept rank and the group takes
            // its decision from LDS (waves reading it on their own could see
            // different values and part at the next barrier).
            if (g.rank == 0)
                h.stop = __hip_atomic_load(&A.min_accept[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < r0 + b0;
            g.sync();
            // (lane 0 rewrites h.stop only after the pass's barriers, which
            // every lane reaches after this read)
            if (h.stop) break;
        }
        const uint32_t kmax = min((uint32_t)kXY, k - b0);
        // the pass's conditioning variables: rank r0 + b0 + i (lanes i)
        if (g.rank < (int)kmax) {
            const unsigned long long r = r0 + b0 + (unsigned long long)g.rank;
            const bool sideA = r < rec.nA;
            const int owner = sideA ? rec.i : rec.j;
            const int skip = sideA ? rec.posj : rec.posi;
            const int pos = (int)(sideA ? r : r - rec.nA);
            const int z = A.nbr[P.adj_off + (int64_t)owner * P.n + pos + (pos >= skip ? 1 : 0)];
            PassTest &pt = h.t[g.rank];
            pt.col[2] = P.data + (int64_t)z * P.ld;
            pt.rx = rx;
            pt.ry = ry;
            pt.nz = A.cards[P.var_off + z];
            pt.alpha = P.alpha;
        }
        g.sync();
        uint32_t cells[kXY], marg[kXY];
#pragma unroll
        for (int i = 0; i < kXY; ++i) {
            const uint32_t nz = i < (int)kmax ? uni(h.t[i].nz) : 0u;
            cells[i] = rxy * nz;
            marg[i] = (rx + ry + 1u) * nz;
        }
        int kb, logR;
        pass_plan(cells, marg, (int)kmax, Wt, tab_lo, tile.max_rep_log2, m, g.size, &kb, &logR);
        if (kb == 0) {
            o.err = kDevTableTooLarge;
            return o;
        }
        if (g.rank == 0) pass_layout(h, cells, marg, kb, logR);
        uint32_t rep_words = 0;
#pragma unroll
        for (int i = 0; i < kXY; ++i)
            if (i < kb) rep_words += cells[i] << logR;
        g.sync();
        for (uint32_t i = (uint32_t)g.rank; i < rep_words; i += (uint32_t)g.size) tabs[i] = 0u;
        g.sync();
        count_xy(xc, yc, h, tab_lo, kb, rx, rxy, logR, m, g.rank, g.size);
        g.sync();
        int nflag = 0;
        const bool acc = pass_finish<kGeneral>(g, h, tabs, kb, logR, tile, &nflag);
        if (acc) atomicMin(&h.first, g.rank);
        g.sync();
        const int first = h.first;
        o.exec += (uint32_t)kb;
        o.rechecks += (uint32_t)nflag;
        g.sync();  // the header is rewritten by the next pass
        if (first < kXY) {
            o.first_accept = (int32_t)b0 + first;
            break;
        }
        b0 += (uint32_t)kb;
    }
    return o;
}

static_assert(kGrabParts <= 8, "counter indices are packed into 3 bits");
constexpr int kGrabPartsLog2 = 3;
static_assert(kGrabParts == 1 << kGrabPartsLog2, "a power of two");

// Dynamic units (those from S0 on) are dealt to the counters in blocks of
// 2^lgb consecutive units: the i-th unit of counter p is dyn_unit(S0, p, i, lgb).
BNS_INLINE unsigned long long dyn_unit(unsigned long long S0, int p, unsigned long long i, int lgb) {
    const unsigned long long blk = i >> lgb, off = i - (blk << lgb);
    return S0 + ((blk * kGrabParts + (unsigned long long)p) << lgb) + off;
}
// Units of counter p below `units`.
BNS_INLINE unsigned long long dyn_units(unsigned long long units, unsigned long long S0, int p, int lgb) {
    const unsigned long long D = units > S0 ? units - S0 : 0ull;
    const int lrow = kGrabPartsLog2 + lgb;  // (shifts: no 64-bit division)
    const unsigned long long full = D >> lrow, rem = D - (full << lrow);
    const unsigned long long lo = (unsigned long long)p << lgb;
    const unsigned long long extra = rem > lo ? min(rem - lo, 1ull << lgb) : 0ull;
    return (full << lgb) + extra;
}

BNS_INLINE unsigned long long shfl_xor_u64(unsigned long long v, int off) {
    const unsigned lo = __shfl_xor((unsigned)(v & 0xffffffffull), off, 64);
    const unsigned hi = __shfl_xor((unsigned)(v >> 32), off, 64);
    return ((unsigned long long)hi << 32) | lo;
}

// Values of the group's rank 0 in every lane of the group (a workgroup goes
// through `slot` in LDS).
BNS_INLINE void group_bcast2_u64(const Grp &g, unsigned long long &a, unsigned long long &b,
                                 unsigned long long (&slot)[2]) {
    if (!g.block) {
        a = bcast_u64(a);
        b = bcast_u64(b);
        return;
    }
    if (threadIdx.x == 0) {
        slot[0] = a;
        slot[1] = b;
    }
    __syncthreads();
    a = slot[0];
    b = slot[1];
    __syncthreads();
}

// Header of a depth, read by one thread of each workgroup.
struct TestHdr {
    unsigned long long total, units, cap;
    long long Lc;
    int32_t quit, d, C, mode, B, bstride, brows, xy;
};

// Units of a grab: i0 + r (part < 0: the first, static batch) or
// dyn_unit(S0, part, i0 + r), r < cnt.
struct Batch {
    unsigned long long i0;
    int part, cnt;
};

// LGB: log2 of the run of consecutive units dealt to a grab counter (a
// template parameter: the kernel's registers are tight, and the instance for
// single units keeps the shortest arithmetic).
// VERIFY: the verification instance (every test also evaluated in FP64 and
// its FP32 error logged); the timed searches use the other.
// GENERAL: the instance for other statistics or df rules than G^2 with the
// declared df.
// UNITS: the instance for a depth of (edge, level) units (1, run_xy_unit);
// a separate instance keeps that path's registers out of the per-test one (0).
// 2: the per-test instance for depths up to kNarrowDepth (tests of at most
// four columns), without the wider counting loops (fewer spilled registers).
template <int LGB, bool VERIFY, bool GENERAL, int UNITS = 0>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(3))) void k_depth_tests(DepthArgs A) {
    extern __shared__ uint32_t lds[];
    __shared__ TestSh tsh[kWaves];
    __shared__ Desc slots[kWaves * kSlotsPerWave];
    __shared__ unsigned long long lvl_base[kMaxLevels + 1];
    __shared__ unsigned long long lvl_cnt[kMaxLevels + 1];
    __shared__ uint64_t btab_lds[kBinomLds];
    __shared__ ProbDev probs_sh[kProbsLds];
    __shared__ uint8_t cards_sh[kCardsLds];
    __shared__ TestHdr hdr;
    __shared__ unsigned long long grab2[2];
    // per-group tallies (kept in LDS: no vector registers across tests)
    __shared__ unsigned long long tal_exec[kWaves], tal_re[kWaves];
    __shared__ double tal_bytes[kWaves];
    Ctl *c = A.ctl;
    const unsigned long long t_enter = wall_clock64();
    // Everything the workgroup needs from the control block and the search
    // set-up is loaded in one round: header, level table, binomial slice,
    // problem records and cardinalities.
    if (threadIdx.x == 0) {
        // (a depth whose tests ran through the Gram contraction: nothing to do)
        hdr.quit = (c->done | c->error) != 0 || c->gram_depth == c->depth;
        hdr.d = c->depth;
        hdr.total = c->total_tickets;
        hdr.units = c->total_units;
        hdr.C = c->chunks;
        hdr.Lc = c->chunk_len;
        hdr.cap = c->split_cap;
        hdr.mode = c->mode;
        hdr.B = c->batch;
        hdr.bstride = c->bstride;
        hdr.brows = c->brows;
        hdr.xy = c->xy;
    }
    if (threadIdx.x < kWaves) {
        tal_exec[threadIdx.x] = 0;
        tal_re[threadIdx.x] = 0;
        tal_bytes[threadIdx.x] = 0.0;
    }
    if (threadIdx.x <= kMaxLevels) {
        lvl_base[threadIdx.x] = c->level_base[threadIdx.x];
        lvl_cnt[threadIdx.x] = c->level_cnt[threadIdx.x];
    }
    for (int i = threadIdx.x; i < kBinomLds; i += kWG) btab_lds[i] = c->bslice[i];
    const bool probs_in_lds = A.n_probs <= kProbsLds;
    const bool cards_in_lds = A.n_globals <= kCardsLds;
    if (probs_in_lds && threadIdx.x < (unsigned)A.n_probs) probs_sh[threadIdx.x] = A.probs[threadIdx.x];
    if (cards_in_lds)
        for (int i = threadIdx.x; i < A.n_globals; i += kWG) cards_sh[i] = A.cards[i];
    __syncthreads();
    // (header values are uniform: scalar registers)
    if (uni(hdr.quit)) return;
    const int d = uni(hdr.d);
    // Start of the launch: the entry time of workgroup 0 (dispatched first),
    // a plain store.  (An atomic per workgroup would queue on one address,
    // and a wave's next wait for a load also waits for its older stores.)
    if (blockIdx.x == 0 && threadIdx.x == 0 && d < kMaxDepths) c->stats[d].t_start = t_enter;
    const unsigned long long total = uni(hdr.total);
    const unsigned long long units = uni(hdr.units);
    const int C = uni(hdr.C);
    const long long Lc = uni(hdr.Lc);
    const uint64_t cap = uni(hdr.cap);
    const int mode = uni(hdr.mode);
    if (uni(hdr.xy) != (UNITS == 1 ? 1 : 0) || (UNITS == 2 && d > kNarrowDepth)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) c->error = kDevUnitMismatch;
        return;
    }
    const int B0 = min(max(uni(hdr.B), 1), kSlotsPerWave);
    // binomials C(n, k), n <= max degree, k <= d: from the staged slice when
    // it fits, else from the full table
    const uint64_t *btab = A.binom;
    int bstride = kBinomK, brows = A.binom_rows;
    if (uni(hdr.bstride) > 0) {
        btab = btab_lds;
        bstride = uni(hdr.bstride);
        brows = uni(hdr.brows);
    }
    int nlev = 0;
    while (nlev < kMaxLevels && lvl_cnt[nlev] > 0) ++nlev;
    // (the wave index and every pointer derived from it are wave-uniform:
    // scalar registers, not vector ones)
    const int w = uni((int)(threadIdx.x >> 6));
    // mode 0: one test per wave in a quarter of the LDS; mode 1: one test per
    // workgroup in all of it
    const Grp g = mode ? Grp::workgroup() : Grp::wave();
    TestSh &t = tsh[mode ? 0 : w];
    Desc *mine = mode ? slots : slots + w * kSlotsPerWave;
    const uint32_t W = mode ? (uint32_t)A.tile.lds_words : (uint32_t)A.tile.lds_words / kWaves;
    uint32_t *region = mode ? lds : lds + (uint32_t)w * W;
    const int ti = mode ? 0 : w;  // tally slot of the group
    // Work units: a unit is (ticket, chunk); chunk-major order puts the
    // chunks of one ticket far apart, so they run on different groups at the
    // same time.  Group gid's first batch is units [gid B0, gid B0 + B0),
    // taken without a counter (the grid is launched with exactly G groups);
    // the rest are spread over kGrabParts counters, a workgroup starting on
    // counter blockIdx mod kGrabParts (about one per XCD), so that grabs do
    // not all queue on one address.  Counters deal units in blocks: single
    // units (the finest interleave) when the columns stay in the last-level
    // cache, runs of consecutive tickets (edges that share a column) when
    // they do not, so that each XCD's L2 sees fewer distinct columns.
    const int G = mode ? (int)gridDim.x : (int)gridDim.x * kWaves;
    const int gid = mode ? (int)blockIdx.x : (int)blockIdx.x * kWaves + w;
    const unsigned long long S0 = (unsigned long long)G * (unsigned long long)B0;
    int part = (int)(blockIdx.x % kGrabParts);
    constexpr int lgb = LGB;
    Batch bt;
    bt.i0 = (unsigned long long)gid * (unsigned long long)B0;
    bt.part = -1;
    bt.cnt = bt.i0 < units ? (int)min((unsigned long long)B0, units - bt.i0) : 0;
    unsigned long long left_est = dyn_units(units, S0, part, lgb);  // after the last grab
    for (;;) {
        const int cnt = bt.cnt;
        if (g.rank < cnt) {
            const unsigned long long i = bt.i0 + (unsigned long long)g.rank;
            const unsigned long long u = bt.part < 0 ? i : dyn_unit(S0, bt.part, i, lgb);
            const unsigned long long ch = (C <= 1) ? 0ull
                                          : ((u | total) >> 32) ? u / total
                                                                : (unsigned long long)((uint32_t)u / (uint32_t)total);
            const unsigned long long tk = u - ch * total;
            Desc &q = mine[g.rank];
            decode_ticket(A, lvl_base, lvl_cnt, nlev, tk, d, btab, bstride, brows, C == 1,
                          probs_in_lds ? probs_sh : nullptr, cards_in_lds ? cards_sh : nullptr, q);
            q.tk = tk;
            q.chunk = (int32_t)ch;
        }
        g.sync();
        for (int j = 0; j < cnt; ++j) {
            const Desc &q = mine[j];
            if (!uni(q.valid)) continue;
            if constexpr (UNITS == 1) {
                const XYOut xo = run_xy_unit<GENERAL>(g, region, W, A.tile, A, q);
                if (g.rank == 0) {
                    tal_exec[ti] += xo.exec;
                    tal_re[ti] += xo.rechecks;
                    tal_bytes[ti] += 3.0 * (double)xo.exec * (double)q.m;
                    if (xo.err) c->error = xo.err;
                    if (xo.first_accept >= 0)
                        atomicMin(&A.min_accept[q.e], q.r + (unsigned long long)xo.first_accept);
                    if (A.per_prob && xo.exec) {
                        __hip_atomic_fetch_add(&A.ecnt[2 * (uint64_t)q.e], xo.exec, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                        if (xo.rechecks)
                            __hip_atomic_fetch_add(&A.ecnt[2 * (uint64_t)q.e + 1], xo.rechecks, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                g.sync();
                continue;
            }
            // Lane 0 fetches the next test's current first-accept rank while
            // this test runs and drops that test before it starts if a lower
            // rank of its edge has accepted meanwhile (the check at decode is
            // up to a batch old).  Split depths run every unit.
            const bool chk = C == 1 && j + 1 < cnt && g.rank == 0 && mine[j + 1].valid;
            unsigned long long ma_next = ~0ull;
            if (chk)
                ma_next = __hip_atomic_load(&A.min_accept[mine[j + 1].e], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
            stage_test(g, q, t);
            const int64_t qm = uni(q.m);
            // Split depths: unit (ticket, chunk) counts its chunk of samples
            // into the ticket's merge table; the group that merges the last
            // chunk evaluates the test from the merged table and clears it.
            // A test whose table exceeds the merge table runs whole in chunk 0.
            Src src{nullptr, nullptr, 0, qm};
            uint32_t *gt = nullptr;
            uint32_t nch = 1;
            if (C > 1) {
                const int chunk = uni(q.chunk);
                const int64_t s0 = (int64_t)chunk * Lc;
                nch = (uint32_t)((qm + Lc - 1) / Lc);
                if (nch > 1 && table_cells(t) <= cap) {
                    if (s0 >= qm) continue;
                    gt = A.split_tab + uni(q.tk) * cap;
                    src.gdst = gt;
                    src.s0 = s0;
                    src.s1 = min(qm, s0 + (int64_t)Lc);
                } else if (chunk != 0) {
                    continue;
                }
            }
            for (;;) {
                const TestOut o = run_test<VERIFY, GENERAL, UNITS == 2 ? kNarrowDepth + 2 : kMaxCols>(
                    g, t, region, W, A.tile, uni(q.alpha), nullptr, src);
                if (g.rank == 0) tal_bytes[ti] += (double)q.ncols * (double)(src.s1 - src.s0);
                if (src.gdst) {
                    // Every access to a merge table and its chunk counter is
                    // an agent-scope atomic, so each word has one order of
                    // updates seen by all XCDs.  Each wave of the group has
                    // consumed the values its adds returned, so its adds are
                    // performed before the barrier; the barrier orders them
                    // before rank 0's counter increment, a release at agent
                    // scope.  The group that counts the last chunk acquires
                    // at agent scope with the same increment, and its table
                    // loads come after it: every chunk's adds are visible.
                    g.sync();
                    uint32_t prev = 0;
                    if (g.rank == 0)
                        prev = __hip_atomic_fetch_add(&A.split_cnt[q.tk], 1u, __ATOMIC_ACQ_REL,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                    prev = g.bcast(prev, t);
                    if (prev + 1 != nch) break;
                    // the counter is not touched again in this launch
                    if (g.rank == 0)
                        __hip_atomic_store(&A.split_cnt[q.tk], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    src = Src{gt, nullptr, 0, 0};  // evaluate the merged table
                    continue;
                }
                if (src.gsrc) {
                    // cleared with agent-scope atomic stores (after the last
                    // read of the table, which the FP64 re-check may repeat);
                    // the next use of these words is by a later launch
                    g.sync();
                    const uint32_t T = (uint32_t)table_cells(t);
                    for (uint32_t i = g.rank; i < T; i += g.size)
                        __hip_atomic_store(gt + i, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                if (g.rank == 0) {
                    ++tal_exec[ti];
                    if (o.flags & 2) ++tal_re[ti];
                    if (o.err) c->error = o.err;
                    if (o.flags & 1) atomicMin(&A.min_accept[q.e], q.r);
                    if (VERIFY && !src.gdst) {
                        const unsigned long long k = atomicAdd(A.err_cnt, 1ull);
                        if ((int64_t)k < A.err_cap) {
                            const double ref = o.g2_ref;
                            A.err_val[k] = (float)(fabs(o.g2_first - ref) / fmax(fabs(ref), 1.0));
                            A.err_tag[k] = ((uint32_t)q.prob << 16) | ((uint32_t)o.flip << 8) | (uint32_t)d;
                        }
                    }
                    if (A.per_prob) {
                        __hip_atomic_fetch_add(&A.ecnt[2 * (uint64_t)q.e], 1u, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                        if (o.flags & 2)
                            __hip_atomic_fetch_add(&A.ecnt[2 * (uint64_t)q.e + 1], 1u, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                break;
            }
            if (chk && mine[j + 1].r > ma_next) mine[j + 1].valid = 0;
            g.sync();
        }
        // Next grab: B0 units from the group's counter.  Once that counter
        // is known to be used up, ranks 1..kGrabParts-1 read the other
        // counters in the same round trip, so that the group moves to the one
        // with the most units left, or stops.
        bt.cnt = 0;
        for (;;) {
            const unsigned long long np = dyn_units(units, S0, part, lgb);
            const bool scan = left_est == 0;
            unsigned long long k = 0, key = 0;
            if (g.rank == 0) {
                if (np > 0) k = atomicAdd(&c->grab_ctr[part * kGrabStride], (unsigned long long)B0);
            } else if (scan && g.rank < kGrabParts) {
                const int r = (part + g.rank) % kGrabParts;
                const unsigned long long nr = dyn_units(units, S0, r, lgb);
                if (nr > 0) {
                    const unsigned long long kr = __hip_atomic_load(&c->grab_ctr[r * kGrabStride],
                                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (nr > kr) key = ((nr - kr) << 3) | (unsigned long long)r;
                }
            }
            // the counter with the most units left (ranks 1..kGrabParts-1 are
            // lanes of the group's first wave)
            if (scan && (threadIdx.x < 64 || !g.block)) {
#pragma unroll
                for (int off = 1; off < kGrabParts; off <<= 1) {
                    const unsigned long long o = shfl_xor_u64(key, off);
                    key = o > key ? o : key;
                }
            }
            group_bcast2_u64(g, k, key, grab2);
            k = uni(k);
            key = uni(key);
            if (np > 0 && k < np) {
                bt.i0 = k;
                bt.part = part;
                bt.cnt = (int)min((unsigned long long)B0, np - k);
                left_est = np - k - (unsigned long long)bt.cnt;
                break;
            }
            // the counter is used up: move to the one with the most units
            // left (read with this grab, or with the next one), or stop when
            // none has any
            if (!scan) {
                left_est = 0;
                continue;
            }
            if (key == 0) break;
            part = (int)(key & 7ull);
        }
        if (bt.cnt == 0) break;
    }
    __syncthreads();
    if (threadIdx.x < kWaves && d < kMaxDepths) {
        const int k = threadIdx.x;
        if (tal_exec[k]) atomicAdd(&c->stats[d].executed, tal_exec[k]);
        if (tal_re[k]) atomicAdd(&c->stats[d].rechecks, tal_re[k]);
        if (tal_bytes[k] > 0.0) atomicAdd(&c->stats[d].operand_bytes, tal_bytes[k]);
        if (k == 0) atomicMax(&c->stats[d].t_end, (unsigned long long)wall_clock64());
    }
}

// ---------------------------------------------------------------------------
// Edge-level form (the edge-level parallelism of Section IV-A): a group of
// lanes (a wave, or a workgroup with test_group 2) takes one edge of the
// depth at a time and runs its tests in the sequential order until the first
// accepting one.  No test is speculative, and a group holds an edge for all of
// its tests, so edges with many tests bound the depth's time.
// ---------------------------------------------------------------------------
template <bool GENERAL>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(3))) void k_depth_edges(DepthArgs A) {
    extern __shared__ uint32_t lds[];
    __shared__ TestSh tsh[kWaves];
    __shared__ Desc slots[kWaves];
    __shared__ uint64_t btab_lds[kBinomLds];
    __shared__ ProbDev probs_sh[kProbsLds];
    __shared__ uint8_t cards_sh[kCardsLds];
    __shared__ int hdr[4];
    __shared__ unsigned long long hdr_edges;
    __shared__ unsigned long long grab[2];
    __shared__ unsigned long long tal_exec[kWaves], tal_re[kWaves];
    __shared__ double tal_bytes[kWaves];
    Ctl *c = A.ctl;
    const unsigned long long t_enter = wall_clock64();
    if (threadIdx.x == 0) {
        hdr[0] = (c->done | c->error) != 0;
        hdr[1] = c->depth;
        hdr[2] = c->bstride;
        hdr[3] = c->brows;
        hdr_edges = c->n_edges;
    }
    if (threadIdx.x < kWaves) {
        tal_exec[threadIdx.x] = 0;
        tal_re[threadIdx.x] = 0;
        tal_bytes[threadIdx.x] = 0.0;
    }
    for (int i = threadIdx.x; i < kBinomLds; i += kWG) btab_lds[i] = c->bslice[i];
    const bool probs_in_lds = A.n_probs <= kProbsLds;
    const bool cards_in_lds = A.n_globals <= kCardsLds;
    if (probs_in_lds && threadIdx.x < (unsigned)A.n_probs) probs_sh[threadIdx.x] = A.probs[threadIdx.x];
    if (cards_in_lds)
        for (int i = threadIdx.x; i < A.n_globals; i += kWG) cards_sh[i] = A.cards[i];
    __syncthreads();
    if (uni(hdr[0])) return;
    const int d = uni(hdr[1]);
    const unsigned long long E = uni(hdr_edges);
    if (blockIdx.x == 0 && threadIdx.x == 0 && d < kMaxDepths) c->stats[d].t_start = t_enter;
    const uint64_t *btab = A.binom;
    int bstride = kBinomK, brows = A.binom_rows;
    if (uni(hdr[2]) > 0) {
        btab = btab_lds;
        bstride = uni(hdr[2]);
        brows = uni(hdr[3]);
    }
    const int w = uni((int)(threadIdx.x >> 6));
    const int mode = A.mode_policy == 2 ? 1 : 0;  // one wave per edge unless a workgroup is asked for
    const Grp g = mode ? Grp::workgroup() : Grp::wave();
    TestSh &t = tsh[mode ? 0 : w];
    Desc &q = slots[mode ? 0 : w];
    const uint32_t W = mode ? (uint32_t)A.tile.lds_words : (uint32_t)A.tile.lds_words / kWaves;
    uint32_t *region = mode ? lds : lds + (uint32_t)w * W;
    const int ti = mode ? 0 : w;
    for (;;) {
        unsigned long long e = 0, z = 0;
        if (g.rank == 0) e = atomicAdd(&c->grab_ctr[0], 1ull);
        group_bcast2_u64(g, e, z, grab);
        e = uni(e);
        if (e >= E) break;
        const EdgeRec rec = A.edges[e];
        const unsigned long long n = uni((unsigned long long)rec.n);
        for (unsigned long long r = 0; r < n; ++r) {
            if (g.rank == 0)
                decode_edge_rank(A, (int64_t)e, r, rec, d, btab, bstride, brows, probs_in_lds ? probs_sh : nullptr,
                                 cards_in_lds ? cards_sh : nullptr, q);
            g.sync();
            stage_test(g, q, t);
            const int64_t qm = uni(q.m);
            const TestOut o = run_test<false, GENERAL>(g, t, region, W, A.tile, uni(q.alpha), nullptr,
                                                       Src{nullptr, nullptr, 0, qm});
            const bool accepted = (uni((uint32_t)o.flags) & 1u) != 0;
            if (g.rank == 0) {
                ++tal_exec[ti];
                if (o.flags & 2) ++tal_re[ti];
                tal_bytes[ti] += (double)q.ncols * (double)qm;
                if (o.err) c->error = o.err;
                if (accepted) atomicMin(&A.min_accept[e], r);
                if (A.per_prob) {
                    __hip_atomic_fetch_add(&A.ecnt[2 * e], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (o.flags & 2)
                        __hip_atomic_fetch_add(&A.ecnt[2 * e + 1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            g.sync();
            if (accepted || o.err) break;
        }
    }
    __syncthreads();
    if (threadIdx.x < kWaves && d < kMaxDepths) {
        const int k = threadIdx.x;
        if (tal_exec[k]) atomicAdd(&c->stats[d].executed, tal_exec[k]);
        if (tal_re[k]) atomicAdd(&c->stats[d].rechecks, tal_re[k]);
        if (tal_bytes[k] > 0.0) atomicAdd(&c->stats[d].operand_bytes, tal_bytes[k]);
        if (k == 0) atomicMax(&c->stats[d].t_end, (unsigned long long)wall_clock64());
    }
}

// ---------------------------------------------------------------------------
// Depth completion: remove accepted edges, record sepsets and the canonical
// test count (per edge: ranks up to and including its first accepting one).
// The last block to finish advances the control block to the next depth.
// ---------------------------------------------------------------------------
// Removals of edges [first, E) in steps of stride (per wave): accepted edges
// leave the graph; the canonical test count and removals are tallied into
// req and rem.  Removal records of depth >= 1 go to the pool, densely:
// [problem, i, j, s_1 .. s_d] (d + 3 words), one atomic per wave.
// One edge per lane (all lanes of the wave call it together; valid marks
// the lanes that hold an edge).
// pool_lds (optional): an LDS counter of removal-record words (a removal
// kernel of one workgroup), instead of the control block's.
BNS_INLINE void apply_one(const DepthArgs &A, Ctl *c, int d, bool valid, const EdgeRec &r,
                          unsigned long long ma, unsigned long long &rem, const Binom &bn,
                          const ProbDev *probs, uint64_t *lds_bits, unsigned long long *pool_lds) {
    const int lane = threadIdx.x & 63;
    const uint64_t lt = lanes_below_mask();
    const bool removed = valid && ma != ~0ull;
    const uint64_t rmask = __ballot(removed);
    if (rmask == 0ull) return;
    rem += removed ? 1 : 0;
    unsigned long long off = 0;
    if (d > 0) {
        const unsigned long long rec = (unsigned long long)(d + 3);
        unsigned long long b0 = 0;
        if (lane == 0)
            b0 = atomicAdd(pool_lds ? pool_lds : &c->pool_used, rec * (unsigned long long)__popcll(rmask));
        b0 = __shfl(b0, 0, 64);
        off = b0 + rec * (unsigned long long)__popcll(rmask & lt);
    }
    if (!removed) return;
    const ProbDev &P = probs[r.prob];
    const int n = P.n;
    if (d > 0) {
        int32_t cpos[kMaxZ];
        const bool sideA = ma < r.nA;
        const int owner = sideA ? r.i : r.j;
        const int skip = sideA ? r.posj : r.posi;
        const int64_t p = sideA ? r.pA : r.pB;
        unrank_serial(bn, p, d, sideA ? ma : ma - r.nA, cpos);
        const int32_t *nbo = A.nbr + P.adj_off + (int64_t)owner * n;
        A.pool[off] = r.prob;
        A.pool[off + 1] = r.i;
        A.pool[off + 2] = r.j;
        for (int k = 0; k < d; ++k) {
            const int q = cpos[k];
            A.pool[off + 3 + k] = nbo[q + (q >= skip ? 1 : 0)];
        }
    }
    const int64_t ij = P.adj_off + (int64_t)r.i * n + r.j;
    const int64_t ji = P.adj_off + (int64_t)r.j * n + r.i;
    if (lds_bits) {
        const int W = (n + 63) >> 6;
        uint64_t *rows = lds_bits + P.bit_off;
        atomicAnd(&rows[r.i * W + (r.j >> 6)], ~(1ull << (r.j & 63)));
        atomicAnd(&rows[r.j * W + (r.i >> 6)], ~(1ull << (r.i & 63)));
    } else {
        A.adj[ij] = 0;
        A.adj[ji] = 0;
    }
    A.rdepth[ij] = (int8_t)d;
    A.rdepth[ji] = (int8_t)d;
}

// Per-problem counters of the edges held by the wave's lanes (valid lanes):
// one atomic per distinct problem and counter.
BNS_INLINE void tally_by_problem(const DepthArgs &A, int d, bool valid, int prob, unsigned long long req,
                                 unsigned long long rem, unsigned long long ex, unsigned long long re) {
    if (d >= kMaxDepths) return;
    const int lane = threadIdx.x & 63;
    uint64_t todo = __ballot(valid);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int P = __shfl(prob, leader, 64);
        const bool mine = valid && prob == P;
        const unsigned long long s0 = wave_sum(mine ? req : 0ull);
        const unsigned long long s1 = wave_sum(mine ? rem : 0ull);
        const unsigned long long s2 = wave_sum(mine ? ex : 0ull);
        const unsigned long long s3 = wave_sum(mine ? re : 0ull);
        if (lane == leader) {
            PStatDev &ps = A.pstat[(int64_t)P * kMaxDepths + d];
            if (s0) atomicAdd(&ps.required, s0);
            if (s1) atomicAdd(&ps.removed, s1);
            if (s2) atomicAdd(&ps.executed, s2);
            if (s3) atomicAdd(&ps.rechecks, s3);
        }
        todo &= ~__ballot(mine);
    }
}

BNS_INLINE void apply_edges(const DepthArgs &A, Ctl *c, int d, unsigned long long first,
                            unsigned long long stride, unsigned long long &req,
                            unsigned long long &rem, const Binom &bn, const ProbDev *probs,
                            uint64_t *lds_bits = nullptr, unsigned long long *pool_lds = nullptr,
                            unsigned long long E = ~0ull) {
    if (E == ~0ull) E = c->n_edges;
    const int lane = threadIdx.x & 63;
    // two strides per trip: both edges' loads are in flight together
    for (unsigned long long base = first; base < E; base += 2 * stride) {
        const unsigned long long e0 = base + lane, e1 = base + stride + lane;
        const bool v0 = e0 < E, v1 = e1 < E;
        EdgeRec r0, r1;
        unsigned long long ma0 = ~0ull, ma1 = ~0ull;
        if (v0) {
            r0 = A.edges[e0];
            ma0 = A.min_accept[e0];
        }
        if (v1) {
            r1 = A.edges[e1];
            ma1 = A.min_accept[e1];
        }
        if (v0) req += (ma0 == ~0ull) ? r0.n : ma0 + 1;
        if (v1) req += (ma1 == ~0ull) ? r1.n : ma1 + 1;
        if (A.per_prob) {
            tally_by_problem(A, d, v0, v0 ? r0.prob : 0, v0 ? ((ma0 == ~0ull) ? r0.n : ma0 + 1) : 0ull,
                             (v0 && ma0 != ~0ull) ? 1ull : 0ull, v0 ? A.ecnt[2 * e0] : 0u,
                             v0 ? A.ecnt[2 * e0 + 1] : 0u);
            tally_by_problem(A, d, v1, v1 ? r1.prob : 0, v1 ? ((ma1 == ~0ull) ? r1.n : ma1 + 1) : 0ull,
                             (v1 && ma1 != ~0ull) ? 1ull : 0ull, v1 ? A.ecnt[2 * e1] : 0u,
                             v1 ? A.ecnt[2 * e1 + 1] : 0u);
        }
        apply_one(A, c, d, v0, r0, ma0, rem, bn, probs, lds_bits, pool_lds);
        if (base + stride < E) apply_one(A, c, d, v1, r1, ma1, rem, bn, probs, lds_bits, pool_lds);
    }
}

// Binomials C(n, k), n <= max degree, k <= d, staged in LDS (the unranking
// of a separating set walks them serially); the device table otherwise.
BNS_INLINE Binom stage_binom(const DepthArgs &A, int maxdeg, int d, uint64_t *lds, int cap,
                             int nthreads) {
    const int rows = maxdeg + 1, stride = d + 1;
    if (d > kMaxZ || rows > A.binom_rows || rows * stride > cap)
        return Binom{A.binom, kBinomK, A.binom_rows};
    for (int i = threadIdx.x; i < rows * stride; i += nthreads) {
        const int n = i / stride, k = i - n * stride;
        lds[i] = A.binom[n * kBinomK + k];
    }
    return Binom{lds, stride, rows};
}

// Depth completion over many workgroups; the last one to finish advances
// the control block to the next depth.
__global__ __launch_bounds__(kWG) void k_apply(DepthArgs A) {
    Ctl *c = A.ctl;
    if (c->done) return;
    __shared__ unsigned long long red[2][kWaves];
    __shared__ uint64_t btab[kApplyBinom];
    const int d = c->depth;
    const Binom bn = stage_binom(A, c->maxdeg, d, btab, kApplyBinom, kWG);
    __syncthreads();
    unsigned long long req = 0, rem = 0;
    apply_edges(A, c, d, (unsigned long long)blockIdx.x * kWG + (threadIdx.x & ~63u),
                (unsigned long long)gridDim.x * kWG, req, rem, bn, A.probs);
    req = wave_sum(req);
    rem = wave_sum(rem);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = req;
        red[1][threadIdx.x >> 6] = rem;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, b = 0;
        for (int w = 0; w < kWaves; ++w) {
            a += red[0][w];
            b += red[1][w];
        }
        if (d < kMaxDepths) {
            if (a) atomicAdd(&c->stats[d].required, a);
            if (b) atomicAdd(&c->stats[d].removed, b);
        }
        __threadfence();
        const unsigned int fin = atomicAdd(&c->apply_done, 1u);
        if (fin == gridDim.x - 1) {
            // every block has read the depth: advance to the next one
            c->depth = d + 1;
            c->apply_done = 0;
        }
    }
}

// Small searches: completion of depth d and preparation of depth d + 1 in
// one workgroup (the adjacency updates are visible to the whole workgroup
// after the barrier).
__global__ __launch_bounds__(kSmallThreads) void k_apply_small(DepthArgs A) {
    __shared__ SmallSh sh;
    Ctl *c = A.ctl;
    // One round of loads: control-block header, bit rows, problem records
    // and the depth's binomial slice (staged by the preparation).
    if (threadIdx.x == 0) {
        sh.h_done = c->done;
        sh.h_depth = c->depth;
        sh.h_maxdeg = c->maxdeg;
        sh.h_bstride = c->bstride;
        sh.h_brows = c->brows;
        sh.h_edges = c->n_edges;
        sh.pool_ctr = c->pool_used;
    }
    small_load(A, sh);
    for (int i = threadIdx.x; i < kBinomLds; i += kSmallThreads) sh.btab[i] = c->bslice[i];
    __syncthreads();
    if (sh.h_done) return;
    const int d = sh.h_depth;
    const int w = threadIdx.x >> 6;
    const Binom bn = sh.h_bstride > 0 ? Binom{sh.btab, sh.h_bstride, sh.h_brows}
                                      : Binom{A.binom, kBinomK, A.binom_rows};
    unsigned long long req = 0, rem = 0;
    apply_edges(A, c, d, (unsigned long long)w * 64, (unsigned long long)kSmallThreads, req, rem,
                bn, A.n_probs <= kSmallProbs ? sh.probs : A.probs, sh.bits, &sh.pool_ctr, sh.h_edges);
    req = wave_sum(req);
    rem = wave_sum(rem);
    if ((threadIdx.x & 63) == 0) {
        sh.red[0][w] = req;
        sh.red[1][w] = rem;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, b = 0;
        for (int i = 0; i < kSmallWaves; ++i) {
            a += sh.red[0][i];
            b += sh.red[1][i];
        }
        // (this kernel is the depth's only writer of these: plain stores)
        if (d < kMaxDepths) {
            c->stats[d].required = a;
            c->stats[d].removed = b;
        }
        c->pool_used = sh.pool_ctr;
        c->depth = d + 1;
    }
    // the bit rows after the removals, for the next depth's removal kernel
    for (int i = threadIdx.x; i < A.bit_words; i += kSmallThreads) A.adjbits[i] = sh.bits[i];
    prepare_block(A, c, d + 1, sh);
}

// Copies the control block and, with h_res, the removal depths and the
// removal records written so far (at most res_pool_words) into pinned host
// memory, so that the host reads a launch's results with no copy of its own;
// then raises the completion flag, which the host sees earlier than the
// stream's own completion.
__global__ __launch_bounds__(kWG) void k_publish(DepthArgs A) {
    const int64_t tid = (int64_t)blockIdx.x * kWG + threadIdx.x, nth = (int64_t)gridDim.x * kWG;
    static_assert(sizeof(Ctl) % 16 == 0, "16-byte copies of the control block");
    const uint4 *cs = reinterpret_cast<const uint4 *>(A.ctl);
    uint4 *cd = reinterpret_cast<uint4 *>(A.h_ctl);
    for (int64_t i = tid; i < (int64_t)(sizeof(Ctl) / 16); i += nth) cd[i] = cs[i];
    if (A.h_res) {
        const uint2 *rs = reinterpret_cast<const uint2 *>(A.rdepth);
        uint2 *rd = reinterpret_cast<uint2 *>(A.h_res);
        for (int64_t i = tid; i < A.res_rbytes / 8; i += nth) rd[i] = rs[i];
        const int64_t used = min((int64_t)A.ctl->pool_used, A.res_pool_words);
        int32_t *pd = reinterpret_cast<int32_t *>(A.h_res + A.res_rbytes);
        for (int64_t i = tid; i < used; i += nth) pd[i] = A.pool[i];
    }
    // every wave's copies visible to the host before its workgroup counts
    // itself done; the last workgroup then writes the flag
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int prev = atomicAdd(A.pub_cnt, 1u);
        if (prev + 1u == gridDim.x) {
            __threadfence_system();
            *A.pub_cnt = 0u;
            const unsigned long long v = *A.pub_seq + 1ull;
            *A.pub_seq = v;
            __hip_atomic_store(A.h_flag, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

// ---------------------------------------------------------------------------
// Launchers of the depth pipeline
// ---------------------------------------------------------------------------
static int grid_rows(int n_globals) { return (n_globals + kWaves - 1) / kWaves; }


// Small searches prepare depth 0 here and every later depth in the removal
// kernel of the depth before; larger ones prepare each depth in
// launch_depth_prepare.
hipError_t launch_init_search(const DepthArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_init_search, dim3(64, a.n_probs), dim3(kWG), 0, s, a);
    if (small_search(a)) hipLaunchKernelGGL(k_prepare_small, dim3(1), dim3(kSmallThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_publish(const DepthArgs &a, hipStream_t s) {
    const int64_t words = std::max<int64_t>(a.h_res ? a.res_rbytes / 8 : 0, (int64_t)(sizeof(Ctl) / 16));
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(64, (words + kWG - 1) / kWG));
    hipLaunchKernelGGL(k_publish, dim3(grid), dim3(kWG), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_depth_prepare(const DepthArgs &a, hipStream_t s) {
    if (small_search(a)) return hipSuccess;
    const int gr = grid_rows(a.n_globals);
    hipLaunchKernelGGL(k_snapshot, dim3(gr), dim3(kWG), 0, s, a);
    hipLaunchKernelGGL(k_scan_rows, dim3(1), dim3(kWG), 0, s, a);
    hipLaunchKernelGGL(k_edges, dim3(gr), dim3(kWG), 0, s, a);
    hipLaunchKernelGGL(k_levels, dim3(1), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_scatter, dim3(a.edge_grid), dim3(kWG), 0, s, a);
    return hipGetLastError();
}

// Instance for the search: tickets dealt in runs when its columns exceed the
// last-level cache's share (grab_block_log2 = kGrabRunLog2), else singly.
static auto depth_tests_kernel(const DepthArgs &a, int units) -> decltype(&k_depth_tests<0, false, false>) {
    const bool general = a.tile.stat != 0 || a.tile.df_rule != 0;
    if (units == 1) {
        if (general) return &k_depth_tests<0, false, true, 1>;
        return a.grab_block_log2 ? &k_depth_tests<kGrabRunLog2, false, false, 1> : &k_depth_tests<0, false, false, 1>;
    }
    if (units == 2 && !general && !a.err_val)
        return a.grab_block_log2 ? &k_depth_tests<kGrabRunLog2, false, false, 2> : &k_depth_tests<0, false, false, 2>;
    // verification and other statistics: single-ticket dealing (the dealing
    // never changes results)
    if (a.err_val) return general ? &k_depth_tests<0, true, true> : &k_depth_tests<0, true, false>;
    if (general) return &k_depth_tests<0, false, true>;
    return a.grab_block_log2 ? &k_depth_tests<kGrabRunLog2, false, false> : &k_depth_tests<0, false, false>;
}

hipError_t launch_depth_tests(const DepthArgs &a, int grid, hipStream_t s, hipEvent_t start,
                              hipEvent_t stop, int units) {
    auto kern = depth_tests_kernel(a, units);
    if (a.edge_form) kern = (a.tile.stat != 0 || a.tile.df_rule != 0) ? &k_depth_edges<true> : &k_depth_edges<false>;
    if (start && stop)
        hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kWG), (size_t)a.tile.lds_words * 4u, s, start, stop, 0, a);
    else
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kWG), (size_t)a.tile.lds_words * 4u, s, a);
    return hipGetLastError();
}

hipError_t launch_depth_apply(const DepthArgs &a, hipStream_t s) {
    if (small_search(a)) hipLaunchKernelGGL(k_apply_small, dim3(1), dim3(kSmallThreads), 0, s, a);
    else hipLaunchKernelGGL(k_apply, dim3(a.edge_grid), dim3(kWG), 0, s, a);
    return hipGetLastError();
}

hipError_t allow_dynamic_lds(int bytes) {
    const void *fns[] = {(const void *)k_depth_tests<kGrabRunLog2, false, false>,
                         (const void *)k_depth_tests<0, false, false>, (const void *)k_depth_tests<0, true, false>,
                         (const void *)k_depth_tests<0, false, true>, (const void *)k_depth_tests<0, true, true>,
                         (const void *)k_depth_tests<0, false, false, 1>,
                         (const void *)k_depth_tests<kGrabRunLog2, false, false, 1>,
                         (const void *)k_depth_tests<0, false, true, 1>,
                         (const void *)k_depth_tests<0, false, false, 2>,
                         (const void *)k_depth_tests<kGrabRunLog2, false, false, 2>,
                         (const void *)k_depth_edges<false>, (const void *)k_depth_edges<true>};
    hipError_t e = hipSuccess;
    for (const void *f : fns)
        if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_ci_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                                bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_plain_count,
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    return e;
}

int depth_tests_max_wg_per_cu(int lds_bytes) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_depth_tests<0, false, false>, kWG, (size_t)lds_bytes) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

int depth_tests_fit_lds(int lds_per_cu) {
    // The workgroups per compute unit that the registers allow, then the
    // dynamic LDS that leaves each of them a share of the compute unit's LDS
    // rounded down to 2 KB: the LDS is allocated in granules, so a share
    // sized to the byte can cost a workgroup per compute unit.
    const int target = depth_tests_max_wg_per_cu(4096);
    hipFuncAttributes fa;
    int stat = 16384;
    if (hipFuncGetAttributes(&fa, (const void *)k_depth_tests<0, false, false>) == hipSuccess) stat = (int)fa.sharedSizeBytes;
    if (lds_per_cu <= 0) lds_per_cu = 65536;
    const int share = (lds_per_cu / max(target, 1)) & ~2047;
    int b = (share - stat) & ~255;
    while (b > 4096 && depth_tests_max_wg_per_cu(b) < target) b -= 256;
    return max(b, 4096);
}

// ---------------------------------------------------------------------------
// Batched CI tests (bns_ci_batch): one test per wave, same device path as the
// skeleton search.
// ---------------------------------------------------------------------------
// Results go to out (one record per test) or, with out null, to the
// separate arrays of soa (any may be null).
__global__ __launch_bounds__(kWG) void k_ci_batch(const uint8_t *data, int64_t ld, int64_t m,
                                                  const uint8_t *cards, const CiTestDev *tests,
                                                  const int32_t *zpool, int64_t n_tests,
                                                  double alpha, Tile tile, CiOutDev *out,
                                                  CiOutSoa soa, uint32_t *tables,
                                                  const int64_t *table_off) {
    extern __shared__ uint32_t lds[];
    __shared__ TestSh tsh[kWaves];
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    TestSh &t = tsh[w];
    const Grp gw = Grp::wave();
    const uint32_t W = (uint32_t)tile.lds_words / kWaves;
    uint32_t *region = lds + (uint32_t)w * W;
    for (int64_t ti = (int64_t)blockIdx.x * kWaves + w; ti < n_tests;
         ti += (int64_t)gridDim.x * kWaves) {
        const CiTestDev q = tests[ti];
        for (int k = lane; k < q.nz + 2; k += 64) {
            const int var = (k == 0) ? q.x : (k == 1) ? q.y : zpool[q.zoff + k - 2];
            t.col[k] = data + (int64_t)var * ld;
            t.card[k] = cards[var];
        }
        gw.sync();
        if (lane == 0) {
            t.ncols = q.nz + 2;
            t.m = m;
            uint32_t mlt = 1;
            for (int k = 0; k < t.ncols; ++k) {
                t.mult[k] = mlt;
                mlt *= t.card[k];
            }
        }
        gw.sync();
        const TestOut o =
            run_test(gw, t, region, W, tile, alpha, tables ? tables + table_off[ti] : nullptr,
                     Src{nullptr, nullptr, 0, m});
        if (lane == 0) {
            CiOutDev r;
            r.g2 = o.g2;
            r.p = o.p;
            r.df = o.df;
            r.flags = o.flags | (o.err ? (o.err << 8) : 0);
            r.pad = 0;
            if (out) {
                out[ti] = r;
            } else {
                if (soa.g2) soa.g2[ti] = r.g2;
                if (soa.p) soa.p[ti] = r.p;
                if (soa.df) soa.df[ti] = r.df;
                if (soa.flags) soa.flags[ti] = r.flags;
            }
        }
        gw.sync();
    }
}

hipError_t launch_ci_batch(const uint8_t *data, int64_t ld, int64_t m, const uint8_t *cards,
                           const CiTestDev *tests, const int32_t *zpool, int64_t n_tests,
                           double alpha, Tile tile, CiOutDev *out, uint32_t *tables,
                           const int64_t *table_off, int grid, hipStream_t s, CiOutSoa soa) {
    hipLaunchKernelGGL(k_ci_batch, dim3(grid), dim3(kWG), (size_t)tile.lds_words * 4u, s, data, ld,
                       m, cards, tests, zpool, n_tests, alpha, tile, out, soa, tables, table_off);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Plain per-test form: the samples of one test spread over the grid (the
// sample-level parallelism of Section IV-A), per-block partial tables in
// global memory, then one workgroup sums them in block order.
// ---------------------------------------------------------------------------
__device__ inline void fill_plain(TestSh &t, const uint8_t *data, int64_t ld, int64_t m,
                                  const uint8_t *cards, const PlainTest &pt) {
    if (threadIdx.x < pt.ncols) {
        const int var = pt.vars[threadIdx.x];
        t.col[threadIdx.x] = data + (int64_t)var * ld;
        t.card[threadIdx.x] = cards[var];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        t.ncols = pt.ncols;
        t.m = m;
        uint32_t mlt = 1;
        for (int k = 0; k < t.ncols; ++k) {
            t.mult[k] = mlt;
            mlt *= t.card[k];
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(kWG) void k_plain_count(const uint8_t *data, int64_t ld, int64_t m,
                                                     const uint8_t *cards, const PlainTest pt,
                                                     int64_t spb, uint32_t *partials, int64_t T,
                                                     int lds_words) {
    extern __shared__ uint32_t lds[];
    __shared__ TestSh t;
    fill_plain(t, data, ld, m, cards, pt);
    const int64_t s0 = (int64_t)blockIdx.x * spb;
    const int64_t s1 = min(m, s0 + spb);
    uint32_t *out = partials + (int64_t)blockIdx.x * T;
    // cell ranges of at most cap cells, followed by one spill word per lane
    const int64_t cap = (int64_t)lds_words - kWG;
    for (int64_t cb = 0; cb < T; cb += cap) {
        const uint32_t Tc = (uint32_t)min(cap, T - cb);
        for (uint32_t i = threadIdx.x; i < Tc + kWG; i += kWG) lds[i] = 0u;
        __syncthreads();
        if (s0 < s1) {
            if (T <= cap)
                count_range<false>(t, lds, 0, Tc, 0, 0, s0, s1, threadIdx.x, kWG);
            else
                count_range<true>(t, lds, (uint32_t)cb, Tc, Tc, 0, s0, s1, threadIdx.x, kWG);
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < Tc; i += kWG) out[cb + i] = lds[i];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kWG) void k_plain_finish(const uint8_t *cards, const PlainTest pt,
                                                      int nblocks, const uint32_t *partials,
                                                      int64_t T, uint32_t *ws, double alpha,
                                                      int stat, int df_rule, CiOutDev *out) {
    __shared__ TestSh t;
    const uint32_t rx = cards[pt.vars[0]], ry = cards[pt.vars[1]];
    uint32_t Z = 1;
    for (int k = 2; k < pt.ncols; ++k) Z *= cards[pt.vars[k]];
    for (int64_t cidx = threadIdx.x; cidx < T; cidx += kWG) {
        uint32_t s = 0;
        for (int b = 0; b < nblocks; ++b) s += partials[(int64_t)b * T + cidx];
        ws[cidx] = s;
    }
    __syncthreads();
    uint32_t *rows = ws + T, *cols = rows + rx * Z, *strata = cols + ry * Z;
    const Grp gb = Grp::workgroup();
    marginals(gb, ws, rows, cols, strata, rx, ry, Z);
    const double part = stat_partial<double>(gb, ws, rows, cols, strata, rx, ry, Z, stat);
    const double g2 = (stat ? 1.0 : 2.0) * gb.sum(part, t);
    int64_t df = (int64_t)(rx - 1) * (int64_t)(ry - 1) * (int64_t)Z;
    if (df_rule) df = (int64_t)gb.sum(adj_df_partial(gb, rows, cols, strata, rx, ry, Z), t);
    const double p = group_tail(gb, df, g2, t).p;
    if (threadIdx.x == 0) {
        CiOutDev r;
        r.g2 = g2;
        r.df = df;
        r.p = p;
        r.flags = (r.p > alpha) ? 1 : 0;
        r.pad = 0;
        *out = r;
    }
}

hipError_t launch_plain_count(const uint8_t *data, int64_t ld, int64_t m, const uint8_t *cards,
                              const PlainTest &t, int64_t spb, int nblocks, uint32_t *partials,
                              int64_t T, int lds_words, hipStream_t s) {
    hipLaunchKernelGGL(k_plain_count, dim3(nblocks), dim3(kWG), (size_t)lds_words * 4u, s, data, ld,
                       m, cards, t, spb, partials, T, lds_words);
    return hipGetLastError();
}

hipError_t launch_plain_finish(const uint8_t *cards, const PlainTest &t, int nblocks,
                               const uint32_t *partials, int64_t T, uint32_t *ws, double alpha,
                               int stat, int df_rule, CiOutDev *out, hipStream_t s) {
    hipLaunchKernelGGL(k_plain_finish, dim3(1), dim3(kWG), 0, s, cards, t, nblocks, partials, T, ws,
                       alpha, stat, df_rule, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Value-range check of device-resident data.
// ---------------------------------------------------------------------------
__global__ void k_validate(const uint8_t *data, int64_t ld, int64_t m, int32_t n,
                           const uint8_t *cards, unsigned long long *bad) {
    const int v = blockIdx.y;
    const uint8_t r = cards[v];
    const uint8_t *col = data + (int64_t)v * ld;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < m;
         s += (int64_t)gridDim.x * blockDim.x) {
        if (col[s] >= r) atomicMin(bad, (unsigned long long)((int64_t)v * m + s));
    }
}

hipError_t launch_validate(const uint8_t *data, int64_t ld, int64_t m, int32_t n,
                           const uint8_t *cards, unsigned long long *bad, hipStream_t s) {
    int64_t gx64 = (m + kWG - 1) / kWG;
    int gx = (int)(gx64 < 64 ? gx64 : 64);
    if (gx < 1) gx = 1;
    hipLaunchKernelGGL(k_validate, dim3(gx, n), dim3(kWG), 0, s, data, ld, m, n, cards, bad);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// LDS increment throughput (a reference for reports on the counting step,
// not part of the search): every lane adds 1 to words of an LDS table,
// sixteen increments per step, the lanes of a wave on different words
// (word = cell * 64 + lane, as the lane-interleaved replicas of a table).
// ---------------------------------------------------------------------------
constexpr int kRateWords = 8192;

__global__ __launch_bounds__(kWG) void k_lds_rate(int steps, unsigned int *sink) {
    __shared__ uint32_t tab[kRateWords];
    for (int i = threadIdx.x; i < kRateWords; i += kWG) tab[i] = 0u;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t a[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const uint32_t h = (threadIdx.x * 2654435761u) ^ ((uint32_t)u * 40503u) ^ (blockIdx.x * 97u);
        a[u] = (((h >> 7) & 63u) << 6) | lane;
    }
    const uint32_t base = lds_offset(tab);
    for (int it = 0; it < steps; ++it) {
        const uint32_t off = ((uint32_t)it << 6) & (kRateWords - 1);
#pragma unroll
        for (int u = 0; u < 16; ++u) lds_inc(base + 4u * ((a[u] + off) & (kRateWords - 1)));
    }
    __syncthreads();
    // the table's total (every increment) leaves the kernel, once per wave
    unsigned long long s = 0;
    for (int i = threadIdx.x; i < kRateWords; i += kWG) s += tab[i];
    s = wave_sum(s);
    if (lane == 0) atomicAdd(sink, (unsigned int)s);
}

hipError_t launch_lds_rate(int grid, int steps, unsigned int *sink, hipStream_t s) {
    hipLaunchKernelGGL(k_lds_rate, dim3(grid), dim3(kWG), 0, s, steps, sink);
    return hipGetLastError();
}

}  // namespace bns
