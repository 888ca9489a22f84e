// gfx950 kernels of the batched G^2 CI-test engine and of the per-depth
// PC-stable pipeline (Algorithm 1; grouping, lexicographic conditioning sets
// and depth-0 handling of Sections IV-B and IV-C).
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
__device__ inline void unrank_serial(const uint64_t *B, int rows, int64_t p, int d, uint64_t rr,
                                     int32_t *c) {
    int64_t x0 = 0;
    for (int k = 0; k < d; ++k) {
        const int j = d - k - 1;
        const uint64_t base = binom_at(B, rows, p - x0, j + 1);
        int64_t x = x0;
        // S(x) = number of subsets (with the current prefix) whose k-th element is < x
        //      = C(p - x0, j + 1) - C(p - x, j + 1)   (hockey-stick identity)
        while (x + 1 <= p - j - 1 && base - binom_at(B, rows, p - (x + 1), j + 1) <= rr) ++x;
        c[k] = (int32_t)x;
        rr -= base - binom_at(B, rows, p - x, j + 1);
        x0 = x + 1;
    }
}

// The same search with the 64 lanes of a wave testing 64 candidate positions
// at once; every lane returns the same c[0..d) (written by lane 0 into c).
__device__ inline void unrank_wave(const uint64_t *B, int rows, int64_t p, int d, uint64_t rr,
                                   int32_t *c) {
    const int lane = threadIdx.x & 63;
    int64_t x0 = 0;
    for (int k = 0; k < d; ++k) {
        const int j = d - k - 1;
        const int64_t xmax = p - j - 1;
        const uint64_t base = binom_at(B, rows, p - x0, j + 1);
        int64_t ck = x0;
        for (int64_t xs = x0;; xs += 64) {
            const int64_t x = xs + lane;
            const bool ok = (x <= xmax) && (base - binom_at(B, rows, p - x, j + 1) <= rr);
            const uint64_t mask = __ballot(ok);
            const int cnt = __popcll(mask);
            if (cnt < 64 || xs + 63 >= xmax) {
                ck = xs + cnt - 1;
                break;
            }
        }
        if (lane == 0) c[k] = (int32_t)ck;
        rr -= base - binom_at(B, rows, p - ck, j + 1);
        x0 = ck + 1;
    }
}

__global__ void k_ci_batch(const uint8_t *data, int64_t ld, int64_t m, const uint8_t *cards,
                           const CiTestDev *tests, const int32_t *zpool, int64_t n_tests,
                           double alpha, Tile tile, CiOutDev *out, uint32_t *tables,
                           const int64_t *table_off);
struct PlainTest;
__global__ void k_plain_count(const uint8_t *data, int64_t ld, int64_t m, const uint8_t *cards,
                              const PlainTest pt, int64_t spb, uint32_t *partials, int64_t T,
                              int lds_words);

// ---------------------------------------------------------------------------
// Search initialisation: complete graph, no removals, control block reset.
// ---------------------------------------------------------------------------
__global__ void k_init_search(DepthArgs A) {
    const int pi = blockIdx.y;
    const ProbDev P = A.probs[pi];
    const int64_t nn = (int64_t)P.n * P.n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / P.n, j = e - i * P.n;
        A.adj[P.adj_off + e] = (i != j) ? 1 : 0;
        A.rdepth[P.adj_off + e] = -1;
        A.sepoff[P.adj_off + e] = -1;
    }
    if (pi == 0 && blockIdx.x == 0) {
        Ctl *c = A.ctl;
        if (threadIdx.x == 0) {
            c->depth = 0;
            c->done = 0;
            c->error = 0;
            c->n_edges = 0;
            c->total_tickets = 0;
            c->ticket_ctr = 0;
            c->pool_used = 0;
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
__global__ __launch_bounds__(kWG) void k_snapshot(DepthArgs A) {
    if (A.ctl->done) return;
    const int g = blockIdx.x * kWaves + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= A.n_globals) return;
    const ProbDev &P = A.probs[A.var2prob[g]];
    const int v = g - P.var_off, n = P.n;
    const uint8_t *row = A.adj + P.adj_off + (int64_t)v * n;
    int32_t *nb = A.nbr + P.adj_off + (int64_t)v * n;
    const uint64_t lt = lanes_below_mask();
    int cnt = 0, hi = 0;
    for (int u0 = 0; u0 < n; u0 += 64) {
        const int u = u0 + lane;
        const bool a = (u < n) && row[u];
        const uint64_t mask = __ballot(a);
        if (a) nb[cnt + __popcll(mask & lt)] = u;
        cnt += __popcll(mask);
        hi += __popcll(__ballot(a && u > v));
    }
    if (lane == 0) {
        A.deg[g] = cnt;
        A.rowcnt[g] = hi;
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
    int64_t s = 0;
    for (int i = b; i < e; ++i) s += A.rowcnt[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int i = 0; i < kWG; ++i) {
            const int64_t v = part[i];
            part[i] = acc;
            acc += v;
        }
        c->n_edges = (unsigned long long)acc;
        c->ticket_ctr = 0;
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
__global__ __launch_bounds__(kWG) void k_edges(DepthArgs A) {
    __shared__ unsigned int hist[kMaxLevels + 2];
    Ctl *c = A.ctl;
    const bool live = !c->done;
    for (int i = threadIdx.x; i < kMaxLevels + 2; i += kWG) hist[i] = 0;
    __syncthreads();
    const int g = blockIdx.x * kWaves + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (live && g < A.n_globals && A.rowcnt[g] > 0) {
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
                e.posi = 0;
                if (nB > 0) {
                    // position of v in the ascending list a(u)
                    const int32_t *nbu = A.nbr + P.adj_off + (int64_t)u * n;
                    int lo = 0, hi2 = du;
                    while (lo < hi2) {
                        const int mid = (lo + hi2) >> 1;
                        if (nbu[mid] < v) lo = mid + 1; else hi2 = mid;
                    }
                    e.posi = lo;
                }
                e.levels = ntot ? 64 - __clzll(ntot) : 0;
                atomicAdd(&hist[e.levels], 1u);
                A.edges_tmp[base + hi + __popcll(mhi & lt)] = e;
            }
            cnt += __popcll(mask);
            hi += __popcll(mhi);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kMaxLevels + 2; i += kWG)
        if (hist[i]) atomicAdd(&c->hist[i], hist[i]);
}

// Single thread: ticket levels.  Edges are ordered by their number of levels,
// descending, so the edges with a test of rank r form a prefix; level L holds
// ranks [2^L - 1, 2^(L+1) - 1) of the first level_cnt[L] edges, rank-major.
__global__ void k_levels(DepthArgs A) {
    Ctl *c = A.ctl;
    if (threadIdx.x != 0 || c->done) return;
    unsigned int acc = 0;
    for (int lv = kMaxLevels + 1; lv >= 0; --lv) {
        c->cursor[lv] = acc;
        acc += c->hist[lv];
    }
    unsigned long long base = 0;
    for (int L = 0; L <= kMaxLevels; ++L) {
        const unsigned long long cnt = (L < kMaxLevels) ? c->cursor[L] : 0ull;
        c->level_base[L] = base;
        c->level_cnt[L] = cnt;
        if (cnt) {
            if (L >= 60 || cnt > ((1ull << 61) >> L)) {
                c->error = kDevTooManyTests;
                break;
            }
            base += cnt << L;
        }
    }
    const int d = c->depth;
    c->total_tickets = base;
    c->ticket_ctr = 0;
    if (base == 0) {
        c->done = 1;
    } else if (d < kMaxDepths) {
        c->stats[d].edges = c->n_edges;
        c->stats[d].tickets = base;
    }
}

// Scatter into level order and reset the per-edge first-accept ranks.
__global__ __launch_bounds__(kWG) void k_scatter(DepthArgs A) {
    Ctl *c = A.ctl;
    if (c->done) return;
    const unsigned long long E = c->n_edges;
    for (unsigned long long e = (unsigned long long)blockIdx.x * kWG + threadIdx.x; e < E;
         e += (unsigned long long)gridDim.x * kWG) {
        const EdgeRec r = A.edges_tmp[e];
        const unsigned int pos = atomicAdd(&c->cursor[r.levels], 1u);
        A.edges[pos] = r;
        A.min_accept[pos] = ~0ull;
    }
}

// ---------------------------------------------------------------------------
// Persistent per-depth test kernel.
//
// Workgroups take tickets from one counter.  A ticket names (edge, rank r);
// the conditioning set is unranked on the fly from r (Section IV-C) over the
// frozen adjacency list of side A (lower id) for r < nA, else side B.  A test
// whose rank exceeds the smallest accepting rank already found for its edge
// is skipped; since every rank below the final smallest accepting rank is
// always run, the edge's first accepting set in the sequential order is found
// exactly, whatever the interleaving.
// ---------------------------------------------------------------------------
struct TicketSh {
    unsigned long long level_base[kMaxLevels + 1];
    unsigned long long level_cnt[kMaxLevels + 1];
    unsigned long long ticket;
    unsigned long long r;
    int64_t edge;
    int32_t go;
    int32_t nlev;
    int32_t pos[kMaxZ];
};

__global__ __launch_bounds__(kWG) void k_depth_tests(DepthArgs A) {
    extern __shared__ uint32_t lds[];
    __shared__ TestSh t;
    __shared__ TicketSh ts;
    Ctl *c = A.ctl;
    if (c->done || c->error) return;
    const int d = c->depth;
    const unsigned long long total = c->total_tickets;
    if (threadIdx.x <= kMaxLevels) {
        ts.level_base[threadIdx.x] = c->level_base[threadIdx.x];
        ts.level_cnt[threadIdx.x] = c->level_cnt[threadIdx.x];
    }
    if (threadIdx.x == 0) {
        int nl = 0;
        while (nl < kMaxLevels && c->level_cnt[nl] > 0) ++nl;
        ts.nlev = nl;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const bool wave0 = threadIdx.x < 64;
    unsigned long long executed = 0, rechecks = 0;
    double bytes = 0.0;
    for (;;) {
        if (threadIdx.x == 0) ts.ticket = atomicAdd(&c->ticket_ctr, 1ull);
        __syncthreads();
        const unsigned long long tk = ts.ticket;
        if (tk >= total) break;
        if (wave0) {
            // level of the ticket: largest L with level_base[L] <= tk
            const bool le = lane < ts.nlev && ts.level_base[lane] <= tk;
            const int L = __popcll(__ballot(le)) - 1;
            const unsigned long long off = tk - ts.level_base[L];
            const unsigned long long cnt = ts.level_cnt[L];
            const unsigned long long jj = off / cnt;
            const int64_t e = (int64_t)(off - jj * cnt);
            const unsigned long long r = ((1ull << L) - 1ull) + jj;
            const EdgeRec rec = A.edges[e];
            const unsigned long long ma =
                __hip_atomic_load(&A.min_accept[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const bool go = (r < rec.n) && (r <= ma);
            if (go) {
                const ProbDev &P = A.probs[rec.prob];
                const int n = P.n;
                const bool sideA = r < rec.nA;
                const int owner = sideA ? rec.i : rec.j;
                const int skip = sideA ? rec.posj : rec.posi;
                const int64_t p = (int64_t)A.deg[P.var_off + owner] - 1;
                if (d > 0)
                    unrank_wave(A.binom, A.binom_rows, p, d, sideA ? r : r - rec.nA, ts.pos);
                // columns: x = V_i, y = V_j, then the conditioning variables
                const int32_t *nbo = A.nbr + P.adj_off + (int64_t)owner * n;
                for (int k = lane; k < d + 2; k += 64) {
                    int var;
                    if (k == 0) var = rec.i;
                    else if (k == 1) var = rec.j;
                    else {
                        const int q = ts.pos[k - 2];
                        var = nbo[q + (q >= skip ? 1 : 0)];
                    }
                    t.col[k] = P.data + (int64_t)var * P.ld;
                    t.card[k] = A.cards[P.var_off + var];
                }
                if (lane == 0) {
                    t.ncols = d + 2;
                    t.m = P.m;
                    ts.r = r;
                    ts.edge = e;
                    t.bcast_d[0] = P.alpha;
                }
            }
            if (lane == 0) ts.go = go ? 1 : 0;
        }
        __syncthreads();
        if (ts.go) {
            if (threadIdx.x == 0) {
                uint32_t mlt = 1;
                for (int k = 0; k < t.ncols; ++k) {
                    t.mult[k] = mlt;
                    mlt *= t.card[k];
                }
            }
            __syncthreads();
            const double alpha = t.bcast_d[0];
            const int64_t e = ts.edge;
            const unsigned long long r = ts.r;
            __syncthreads();
            const TestOut o = run_test(t, lds, A.tile, alpha, nullptr);
            if (threadIdx.x == 0) {
                ++executed;
                bytes += (double)t.ncols * (double)t.m;
                if (o.flags & 2) ++rechecks;
                if (o.err) c->error = o.err;
                if (o.flags & 1) atomicMin(&A.min_accept[e], r);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && d < kMaxDepths) {
        atomicAdd(&c->stats[d].executed, executed);
        atomicAdd(&c->stats[d].rechecks, rechecks);
        atomicAdd(&c->stats[d].operand_bytes, bytes);
    }
}

// ---------------------------------------------------------------------------
// Depth completion: remove accepted edges, record sepsets and the canonical
// test count (per edge: ranks up to and including its first accepting one).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_apply(DepthArgs A) {
    Ctl *c = A.ctl;
    if (c->done) return;
    __shared__ unsigned long long red[2][kWaves];
    const int d = c->depth;
    const unsigned long long E = c->n_edges;
    const unsigned long long pool0 = c->pool_used;
    unsigned long long req = 0, rem = 0;
    for (unsigned long long e = (unsigned long long)blockIdx.x * kWG + threadIdx.x; e < E;
         e += (unsigned long long)gridDim.x * kWG) {
        const EdgeRec r = A.edges[e];
        const unsigned long long ma = A.min_accept[e];
        if (ma == ~0ull) {
            req += r.n;
            continue;
        }
        req += ma + 1;
        ++rem;
        const ProbDev &P = A.probs[r.prob];
        const int n = P.n;
        const unsigned long long off = pool0 + e * (unsigned long long)d;
        if (d > 0) {
            int32_t cpos[kMaxZ];
            const bool sideA = ma < r.nA;
            const int owner = sideA ? r.i : r.j;
            const int skip = sideA ? r.posj : r.posi;
            const int64_t p = (int64_t)A.deg[P.var_off + owner] - 1;
            unrank_serial(A.binom, A.binom_rows, p, d, sideA ? ma : ma - r.nA, cpos);
            const int32_t *nbo = A.nbr + P.adj_off + (int64_t)owner * n;
            for (int k = 0; k < d; ++k) {
                const int q = cpos[k];
                A.pool[off + k] = nbo[q + (q >= skip ? 1 : 0)];
            }
        }
        const int64_t ij = P.adj_off + (int64_t)r.i * n + r.j;
        const int64_t ji = P.adj_off + (int64_t)r.j * n + r.i;
        A.adj[ij] = 0;
        A.adj[ji] = 0;
        A.rdepth[ij] = d;
        A.rdepth[ji] = d;
        A.sepoff[ij] = (int64_t)off;
        A.sepoff[ji] = (int64_t)off;
    }
    req = wave_sum(req);
    rem = wave_sum(rem);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = req;
        red[1][threadIdx.x >> 6] = rem;
    }
    __syncthreads();
    if (threadIdx.x == 0 && d < kMaxDepths) {
        unsigned long long a = 0, b = 0;
        for (int w = 0; w < kWaves; ++w) {
            a += red[0][w];
            b += red[1][w];
        }
        if (a) atomicAdd(&c->stats[d].required, a);
        if (b) atomicAdd(&c->stats[d].removed, b);
    }
}

__global__ void k_finish_depth(DepthArgs A) {
    Ctl *c = A.ctl;
    if (threadIdx.x != 0 || c->done) return;
    c->pool_used += c->n_edges * (unsigned long long)c->depth;
    c->depth += 1;
}

// ---------------------------------------------------------------------------
// Launchers of the depth pipeline
// ---------------------------------------------------------------------------
static int grid_rows(int n_globals) { return (n_globals + kWaves - 1) / kWaves; }

hipError_t launch_init_search(const DepthArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_init_search, dim3(64, a.n_probs), dim3(kWG), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_depth_prepare(const DepthArgs &a, hipStream_t s) {
    const int gr = grid_rows(a.n_globals);
    hipLaunchKernelGGL(k_snapshot, dim3(gr), dim3(kWG), 0, s, a);
    hipLaunchKernelGGL(k_scan_rows, dim3(1), dim3(kWG), 0, s, a);
    hipLaunchKernelGGL(k_edges, dim3(gr), dim3(kWG), 0, s, a);
    hipLaunchKernelGGL(k_levels, dim3(1), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_scatter, dim3(1024), dim3(kWG), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_depth_tests(const DepthArgs &a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_depth_tests, dim3(grid), dim3(kWG), (size_t)a.tile.lds_words * 4u, s, a);
    return hipGetLastError();
}

hipError_t launch_depth_apply(const DepthArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_apply, dim3(1024), dim3(kWG), 0, s, a);
    hipLaunchKernelGGL(k_finish_depth, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t allow_dynamic_lds(int bytes) {
    hipError_t e = hipFuncSetAttribute((const void *)k_depth_tests,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
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
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_depth_tests, kWG, (size_t)lds_bytes) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

// ---------------------------------------------------------------------------
// Batched CI tests (bns_ci_batch)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_ci_batch(const uint8_t *data, int64_t ld, int64_t m,
                                                  const uint8_t *cards, const CiTestDev *tests,
                                                  const int32_t *zpool, int64_t n_tests,
                                                  double alpha, Tile tile, CiOutDev *out,
                                                  uint32_t *tables, const int64_t *table_off) {
    extern __shared__ uint32_t lds[];
    __shared__ TestSh t;
    for (int64_t ti = blockIdx.x; ti < n_tests; ti += gridDim.x) {
        const CiTestDev q = tests[ti];
        if (threadIdx.x < q.nz + 2) {
            const int k = threadIdx.x;
            const int var = (k == 0) ? q.x : (k == 1) ? q.y : zpool[q.zoff + k - 2];
            t.col[k] = data + (int64_t)var * ld;
            t.card[k] = cards[var];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            t.ncols = q.nz + 2;
            t.m = m;
            uint32_t mlt = 1;
            for (int k = 0; k < t.ncols; ++k) {
                t.mult[k] = mlt;
                mlt *= t.card[k];
            }
        }
        __syncthreads();
        const TestOut o = run_test(t, lds, tile, alpha, tables ? tables + table_off[ti] : nullptr);
        if (threadIdx.x == 0) {
            CiOutDev r;
            r.g2 = o.g2;
            r.p = o.p;
            r.df = o.df;
            r.flags = o.flags | (o.err ? (o.err << 8) : 0);
            r.pad = 0;
            out[ti] = r;
        }
        __syncthreads();
    }
}

hipError_t launch_ci_batch(const uint8_t *data, int64_t ld, int64_t m, const uint8_t *cards,
                           const CiTestDev *tests, const int32_t *zpool, int64_t n_tests,
                           double alpha, Tile tile, CiOutDev *out, uint32_t *tables,
                           const int64_t *table_off, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_ci_batch, dim3(grid), dim3(kWG), (size_t)tile.lds_words * 4u, s, data, ld,
                       m, cards, tests, zpool, n_tests, alpha, tile, out, tables, table_off);
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
    for (int64_t cb = 0; cb < T; cb += lds_words) {
        const uint32_t Tc = (uint32_t)min((int64_t)lds_words, T - cb);
        for (uint32_t i = threadIdx.x; i < Tc; i += kWG) lds[i] = 0u;
        __syncthreads();
        if (s0 < s1) count_samples(t, lds, (uint32_t)cb, Tc, 0, s0, s1);
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < Tc; i += kWG) out[cb + i] = lds[i];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kWG) void k_plain_finish(const uint8_t *cards, const PlainTest pt,
                                                      int nblocks, const uint32_t *partials,
                                                      int64_t T, uint32_t *ws, double alpha,
                                                      CiOutDev *out) {
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
    marginals(ws, rows, cols, strata, rx, ry, Z);
    const double part = g2_partial<double>(ws, rows, cols, strata, rx, ry, Z);
    const double g2 = 2.0 * wg_sum(part, t);
    if (threadIdx.x == 0) {
        const int64_t df = (int64_t)(rx - 1) * (int64_t)(ry - 1) * (int64_t)Z;
        CiOutDev r;
        r.g2 = g2;
        r.df = df;
        r.p = chi2_upper(df, g2);
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
                               CiOutDev *out, hipStream_t s) {
    hipLaunchKernelGGL(k_plain_finish, dim3(1), dim3(kWG), 0, s, cards, t, nblocks, partials, T, ws,
                       alpha, out);
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

}  // namespace bns
