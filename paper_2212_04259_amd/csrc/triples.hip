// Depth 1 of the skeleton search (Algorithm 1 at conditioning sets of one
// variable) as masked Gram contractions on gfx950 int8 MFMA.
//
// A depth-1 test of edge (x, y) conditions on one z taken from the frozen
// neighbours of one endpoint, the owner u of that side (x for the tests of
// side A, y for side B; Section IV-C's grouping).  Let H be the one-hot
// columns H[s][(v, a)] = [X_v(s) = a] of u's neighbours v and m_c the samples
// with X_u = c.  The masked Gram matrix G_c = H^T diag(m_c) H holds
//   G_c[(v, a)][(w, b)] = #{s : X_u = c, X_v = a, X_w = b},
// so the table of the test (u, v | w) is N[c][a][b] = G_c[(v, a)][(w, b)] and
// its marginals are sums of entries: N_u+w[c][b] = G_c[(w, b)][(w, b)],
// N_+vw[a][b] = sum_c G_c[(v, a)][(w, b)], N_++w[b] = sum_c G_c[(w, b)][(w, b)].
// Every depth-1 test is evaluated (none is skipped after an accepting one);
// the edge keeps its lowest accepting rank, which is the first accepting test
// of the sequential order, so the skeleton, sepsets and canonical counts are
// those of Algorithm 1.  The products of 0/1 bytes summed in int32 are exact.
//
// k_tri_plan (one workgroup): each node's frozen degree (from the depth's
// edge records), the one-hot row offsets of its neighbours, its work items
// (T x T tiles of the upper triangle of tile blocks, times groups of up to
// four masks, times sample chunks cut toward a target item count), its first
// test, and the edge record of every (node, neighbour) pair.  A plan beyond
// the tile buffer leaves the depth to the test kernel.
// k_tri_gram: one work item per workgroup at a time (2 x 2 waves, each a 32 x
// 32 MFMA block of the tile).  Per step of 512 samples the raw bytes of each
// variable the tile needs (the neighbours of its row and column blocks, and u)
// are staged once in LDS (double-buffered: the next step's loads are in
// flight during this step's MFMAs); each lane forms its one-hot fragments at
// read time with byte permutes (cardinalities 2..8), and each mask multiplies
// the first operand's fragment bytewise before its MFMA.
// k_tri_reduce: sums a node's sample chunks into the first chunk's slab.
// k_tri_eval: one wave per test (lanes over the table's cells, tables and
// marginals in LDS), 64 tests per batch: the tests of a batch are decoded by
// its lanes together, and each lane evaluates one test's chi-square tail
// and records an acceptance with an atomic minimum of the rank on the edge.
#include <algorithm>

#include "device_ci.h"
#include "gram.h"
#include "kernels.h"

namespace bns {

constexpr int kTriT = 64;              // tile side
constexpr int kPlanThreads = 1024;
constexpr int kTriKS = 512;            // samples per pipeline step
constexpr int kTriRow = kTriKS + 16;   // LDS bytes per staged variable and step
constexpr int kTriSlots = 2 * (kTriT / kTriMinCard + 1) + 1;  // variables of both operands, and u
constexpr int kTriLd = (kTriSlots * (kTriKS / 16) + kGramWG - 1) / kGramWG;  // 16-byte loads per thread per step
constexpr long long kTriMinChunk = 4096;  // smallest sample chunk (a multiple of kTriKS)
constexpr int64_t kTriSlab = (int64_t)kTriCats * kTriT * kTriT;  // int32 per work item
constexpr uint32_t kNoCat = 0x0c0c0c0cu;  // byte-permute selector 12 gives 0: no one-hot bit

// Exclusive prefix of v over the workgroup (kPlanThreads threads); *total
// receives the sum.  sh holds kPlanThreads / 64 + 1 words.
BNS_INLINE long long plan_scan(long long v, long long *sh, long long *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    long long incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const long long o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) sh[w] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long run = 0;
        for (int i = 0; i < kPlanThreads / 64; ++i) {
            const long long t = sh[i];
            sh[i] = run;
            run += t;
        }
        sh[kPlanThreads / 64] = run;
    }
    __syncthreads();
    const long long out = sh[w] + incl - v;
    *total = sh[kPlanThreads / 64];
    __syncthreads();
    return out;
}

__global__ __launch_bounds__(kPlanThreads) void k_tri_plan(DepthArgs A) {
    Ctl *c = A.ctl;
    __shared__ long long sh[kPlanThreads / 64 + 1];
    __shared__ int go;
    __shared__ int nch_max;
    const unsigned long long t_enter = wall_clock64();
    if (threadIdx.x == 0) {
        go = (!c->done && c->depth == 1) ? 1 : 0;
        nch_max = 1;
    }
    __syncthreads();
    if (!go) return;
    const TriArgs &X = A.tri;
    const int G = A.n_globals;
    const unsigned long long E = c->n_edges;
    // frozen degrees at depth 1 (nodes without an edge record own no test)
    for (int g = threadIdx.x; g < G; g += kPlanThreads) X.node[g].deg = 0;
    __syncthreads();
    for (unsigned long long e = threadIdx.x; e < E; e += kPlanThreads) {
        const EdgeRec r = A.edges[e];
        const int off = A.probs[r.prob].var_off;
        X.node[off + r.i].deg = r.pA + 1;
        X.node[off + r.j].deg = r.pB + 1;
    }
    __syncthreads();
    // one-hot row offsets, tile blocks and category groups; (tile, group)
    // pairs per node, scanned
    long long carry = 0;
    for (int g0 = 0; g0 < G; g0 += kPlanThreads) {
        const int g = g0 + (int)threadIdx.x;
        long long base = 0;
        if (g < G) {
            TriNode &nd = X.node[g];
            const ProbDev &P = A.probs[A.var2prob[g]];
            const int u = g - P.var_off;
            const int deg = nd.deg;
            const int32_t *nbu = A.nbr + P.adj_off + (int64_t)u * P.n;
            int32_t *ro = X.rowoff + P.adj_off + (int64_t)u * P.n;
            int R = 0;
            for (int k = 0; k < deg; ++k) {
                ro[k] = R;
                R += A.cards[P.var_off + nbu[k]];
            }
            ro[deg] = R;
            nd.R = R;
            nd.nb = (R + kTriT - 1) / kTriT;
            nd.ncg = (A.cards[g] + kTriCats - 1) / kTriCats;
            base = deg >= 2 ? (long long)nd.nb * (nd.nb + 1) / 2 * nd.ncg : 0;
        }
        long long tot = 0;
        const long long pre = plan_scan(base, sh, &tot);
        if (g < G) X.node[g].base_base = carry + pre;
        carry += tot;
    }
    const long long base_total = carry;
    // sample chunks: enough work items to fill the device, each chunk at
    // least kTriMinChunk samples (a multiple of 64)
    const long long full = (A.m_max + kTriKS - 1) / kTriKS * kTriKS;
    long long Lc = full;
    if (base_total > 0 && base_total < (long long)X.target_items) {
        const long long want = ((long long)X.target_items + base_total - 1) / base_total;
        const long long per = (A.m_max + want - 1) / want;
        Lc = (per + kTriKS - 1) / kTriKS * kTriKS;
        if (Lc < kTriMinChunk) Lc = kTriMinChunk;
        if (Lc > full) Lc = full;
    }
    carry = 0;
    for (int g0 = 0; g0 < G; g0 += kPlanThreads) {
        const int g = g0 + (int)threadIdx.x;
        long long items = 0;
        if (g < G) {
            TriNode &nd = X.node[g];
            const ProbDev &P = A.probs[A.var2prob[g]];
            const long long q = (P.m + Lc - 1) / Lc;
            const int nch = q > 1 ? (int)q : 1;
            nd.nch = nch;
            const long long base = nd.deg >= 2 ? (long long)nd.nb * (nd.nb + 1) / 2 * nd.ncg : 0;
            items = base * nch;
            if (items > 0 && nch > 1) atomicMax(&nch_max, nch);
        }
        long long tot = 0;
        const long long pre = plan_scan(items, sh, &tot);
        if (g < G) X.node[g].item_base = carry + pre;
        carry += tot;
    }
    const long long items_total = carry;
    // first test of each node: deg (deg - 1) tests per node
    carry = 0;
    for (int g0 = 0; g0 < G; g0 += kPlanThreads) {
        const int g = g0 + (int)threadIdx.x;
        long long nt = 0;
        if (g < G) {
            const long long dg = X.node[g].deg;
            nt = dg >= 2 ? dg * (dg - 1) : 0;
        }
        long long tot = 0;
        const long long pre = plan_scan(nt, sh, &tot);
        if (g < G) X.node[g].test_base = carry + pre;
        carry += tot;
    }
    const long long tests_total = carry;
    const bool ok = base_total > 0 && items_total <= X.part_items;
    if (ok) {
        // the edge record of every (node, neighbour position)
        for (int g = threadIdx.x; g < G; g += kPlanThreads) {
            const ProbDev &P = A.probs[A.var2prob[g]];
            const int deg = X.node[g].deg;
            int32_t *ei = X.eidx + P.adj_off + (int64_t)(g - P.var_off) * P.n;
            for (int k = 0; k < deg; ++k) ei[k] = -1;
        }
        __syncthreads();
        for (unsigned long long e = threadIdx.x; e < E; e += kPlanThreads) {
            const EdgeRec r = A.edges[e];
            const ProbDev &P = A.probs[r.prob];
            X.eidx[P.adj_off + (int64_t)r.i * P.n + r.posj] = (int32_t)e;
            X.eidx[P.adj_off + (int64_t)r.j * P.n + r.posi] = (int32_t)e;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        c->tri_items = (unsigned long long)items_total;
        c->tri_base = (unsigned long long)base_total;
        c->tri_tests = (unsigned long long)tests_total;
        c->tri_chunk = Lc;
        c->tri_nch_max = nch_max;
        c->gram_depth = ok ? 1 : -1;
        if (ok) {
            c->stats[1].t_start = t_enter;
            c->stats[1].mode = 2;  // a Gram contraction
            c->stats[1].chunks = nch_max;
            c->stats[1].chunk_len = Lc;
        }
    }
}

// One-hot bytes [b == cat] of 16 sample bytes (categories below 8; the byte
// 0x0c, written for samples past a chunk's end, gives 0 for every cat).
BNS_INLINE v4i onehot_perm(const u32x4 &w, uint32_t plo, uint32_t phi) {
    v4i o;
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = (int)__builtin_amdgcn_perm(phi, plo, w[k]);
    return o;
}

BNS_INLINE void cat_pool(uint32_t cat, uint32_t &plo, uint32_t &phi) {
    plo = cat < 4 ? 1u << (8 * cat) : 0u;
    phi = (cat >= 4 && cat < 8) ? 1u << (8 * (cat - 4)) : 0u;
}

// Neighbour index k of one-hot row `row` of a node: ro[k] <= row < ro[k + 1].
BNS_INLINE int row_owner(const int32_t *ro, int deg, int row) {
    int a = 0, z = deg - 1;
    while (a < z) {
        const int mid = (a + z + 1) >> 1;
        if (ro[mid] <= row) a = mid;
        else z = mid - 1;
    }
    return a;
}

__global__ __launch_bounds__(kGramWG) __attribute__((amdgpu_waves_per_eu(2))) void k_tri_gram(DepthArgs A) {
    constexpr int T = kTriT;
    static_assert(T == 64, "one 32 x 32 MFMA block per wave");
    __shared__ __attribute__((aligned(16))) uint8_t raw[2][kTriSlots][kTriRow];  // [buffer][variable][sample]
    __shared__ const uint8_t *slot_col[kTriSlots];
    __shared__ unsigned long long items_sh;
    __shared__ long long chunk_sh;
    __shared__ int quit;
    Ctl *c = A.ctl;
    if (threadIdx.x == 0) {
        quit = (c->done || c->gram_depth != c->depth) ? 1 : 0;
        items_sh = c->tri_items;
        chunk_sh = c->tri_chunk;
    }
    __syncthreads();
    if (quit) return;
    const TriArgs &X = A.tri;
    const unsigned long long nitems = items_sh;
    const long long Lc = chunk_sh;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = w >> 1, wc = w & 1;
    for (unsigned long long item = blockIdx.x; item < nitems; item += gridDim.x) {
        // the node owning the item: the last one whose first item is <= item
        int lo = 0, hi = A.n_globals - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if ((unsigned long long)X.node[mid].item_base <= item) lo = mid;
            else hi = mid - 1;
        }
        const int g = lo;
        const TriNode nd = X.node[g];
        const ProbDev P = A.probs[A.var2prob[g]];
        const int u = g - P.var_off;
        // item -> (tile, category group, chunk)
        const long long rel = (long long)item - nd.item_base;
        const long long bq = rel / nd.nch;
        const int kc = (int)(rel - bq * nd.nch);
        const long long tile = bq / nd.ncg;
        const int cg = (int)(bq - tile * nd.ncg);
        int tr = 0;
        long long rem = tile;
        while (rem >= nd.nb - tr) {
            rem -= nd.nb - tr;
            ++tr;
        }
        const int tc = tr + (int)rem;
        const bool diag = tr == tc;  // the second operand is the first
        const int64_t s0 = (int64_t)kc * Lc;
        const int64_t s1 = min(P.m, s0 + Lc);
        const int nsteps = (int)((s1 - s0 + kTriKS - 1) / kTriKS);
        const int ru = A.cards[g];
        const int c0 = kTriCats * cg;
        const int nc = min(kTriCats, ru - c0);
        const int32_t *nbu = A.nbr + P.adj_off + (int64_t)u * P.n;
        const int32_t *ro = X.rowoff + P.adj_off + (int64_t)u * P.n;
        // staged variables: the neighbours of the row block, then (off the
        // diagonal) those of the column block, then u
        const int kA0 = row_owner(ro, nd.deg, tr * T);
        const int kA1 = row_owner(ro, nd.deg, min(nd.R, tr * T + T) - 1);
        const int kB0 = diag ? kA0 : row_owner(ro, nd.deg, tc * T);
        const int kB1 = diag ? kA1 : row_owner(ro, nd.deg, min(nd.R, tc * T + T) - 1);
        const int nA = kA1 - kA0 + 1;
        const int nB = diag ? 0 : kB1 - kB0 + 1;
        const int nslot = nA + nB + 1;
        if (tid < nslot) {
            const int v = tid < nA ? nbu[kA0 + tid] : tid < nA + nB ? nbu[kB0 + tid - nA] : u;
            slot_col[tid] = P.data + (int64_t)v * P.ld;
        }
        // this lane's fragment rows: (staged variable, category), or none
        int slotA = -1, slotB = -1;
        uint32_t aplo = 0, aphi = 0, bplo = 0, bphi = 0;
        {
            const int row = tr * T + wr * 32 + (lane & 31);
            if (row < nd.R) {
                const int k = row_owner(ro, nd.deg, row);
                slotA = k - kA0;
                cat_pool((uint32_t)(row - ro[k]), aplo, aphi);
            }
            const int col = tc * T + wc * 32 + (lane & 31);
            if (col < nd.R) {
                const int k = row_owner(ro, nd.deg, col);
                slotB = diag ? k - kA0 : nA + k - kB0;
                cat_pool((uint32_t)(col - ro[k]), bplo, bphi);
            }
        }
        uint32_t mplo[kTriCats], mphi[kTriCats];
#pragma unroll
        for (int cc = 0; cc < kTriCats; ++cc) cat_pool((uint32_t)(c0 + cc), mplo[cc], mphi[cc]);
        __syncthreads();  // slot table
        const int slotU = nslot - 1;
        u32x4 pv[kTriLd];
        auto load = [&](int64_t s) {
#pragma unroll
            for (int r = 0; r < kTriLd; ++r) {
                const int id = tid + kGramWG * r;
                const int sl = id >> 5, q = id & 31;
                pv[r] = u32x4{kNoCat, kNoCat, kNoCat, kNoCat};
                if (sl < nslot) {
                    const int64_t ss = s + 16 * q;
                    const int64_t nv = s1 - ss;
                    if (nv > 0) {
                        pv[r] = *(const gvec4 *)(slot_col[sl] + ss);  // (global, not flat)
                        if (nv < 16) {
                            // samples past the chunk's end: no category
#pragma unroll
                            for (int k = 0; k < 4; ++k) {
                                const int64_t vk = nv - 4 * k;
                                const uint32_t keep = vk >= 4 ? 0xffffffffu : vk <= 0 ? 0u : ((1u << (8 * vk)) - 1u);
                                pv[r][k] = (pv[r][k] & keep) | (kNoCat & ~keep);
                            }
                        }
                    }
                }
            }
        };
        auto store = [&](int buf) {
#pragma unroll
            for (int r = 0; r < kTriLd; ++r) {
                const int id = tid + kGramWG * r;
                const int sl = id >> 5, q = id & 31;
                if (sl < nslot) *(u32x4 *)(&raw[buf][sl][16 * q]) = pv[r];
            }
        };
        v16i acc[kTriCats];
#pragma unroll
        for (int cc = 0; cc < kTriCats; ++cc)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[cc][r] = 0;
        load(s0);
        store(0);
        __syncthreads();
        for (int st = 0; st < nsteps; ++st) {
            const int buf = st & 1;
            const bool more = st + 1 < nsteps;
            if (more) load(s0 + (int64_t)(st + 1) * kTriKS);
            // LDS views of the staged rows (LDS reads, not flat ones: a flat
            // read also waits for the step's outstanding global loads)
            typedef __attribute__((address_space(3))) const u32x4 lvec4;
            const uint32_t raw_lo = lds_offset(reinterpret_cast<const uint32_t *>(&raw[buf][0][0]));
            const uint32_t Ra = raw_lo + (uint32_t)(slotA >= 0 ? slotA : 0) * kTriRow;
            const uint32_t Rb = raw_lo + (uint32_t)(slotB >= 0 ? slotB : 0) * kTriRow;
            const uint32_t Ru = raw_lo + (uint32_t)slotU * kTriRow;
#pragma unroll 2
            for (int kk = 0; kk < kTriKS / 32; ++kk) {
                const int koff = 32 * kk + 16 * (lane >> 5);
                const u32x4 wa = *(const lvec4 *)(uintptr_t)(Ra + koff);
                const u32x4 wb = *(const lvec4 *)(uintptr_t)(Rb + koff);
                const u32x4 uw = *(const lvec4 *)(uintptr_t)(Ru + koff);
                const v4i af = slotA >= 0 ? onehot_perm(wa, aplo, aphi) : v4i{0, 0, 0, 0};
                const v4i bf = slotB >= 0 ? onehot_perm(wb, bplo, bphi) : v4i{0, 0, 0, 0};
#pragma unroll
                for (int cc = 0; cc < kTriCats; ++cc) {
                    if (cc >= nc) break;  // uniform
                    const v4i am = af & onehot_perm(uw, mplo[cc], mphi[cc]);
                    acc[cc] = __builtin_amdgcn_mfma_i32_32x32x32_i8(am, bf, acc[cc], 0, 0, 0);
                }
            }
            if (more) store(buf ^ 1);
            __syncthreads();
        }
        // register r of lane l holds row (r % 4) + 4 (l / 32) + 8 (r / 4),
        // column l % 32 of the wave's 32 x 32 block
        int32_t *out = X.part + (int64_t)item * kTriSlab;
#pragma unroll
        for (int cc = 0; cc < kTriCats; ++cc) {
            if (cc >= nc) break;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = wr * 32 + (r & 3) + 4 * (lane >> 5) + 8 * (r >> 2);
                const int col = wc * 32 + (lane & 31);
                out[cc * T * T + row * T + col] = acc[cc][r];
            }
        }
    }
}

// Sums the sample chunks of each (node, tile, category group) into the first
// chunk's slab (coalesced, four entries per lane).
__global__ __launch_bounds__(kWG) void k_tri_reduce(DepthArgs A) {
    Ctl *c = A.ctl;
    if (c->done || c->gram_depth != c->depth || c->tri_nch_max <= 1) return;
    const TriArgs &X = A.tri;
    constexpr int64_t tq = kTriSlab / 4;  // int4 words per slab
    const int64_t total = (int64_t)c->tri_base * tq;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < total; i += (int64_t)gridDim.x * kWG) {
        const int64_t b = i / tq, wd = i - b * tq;
        int lo = 0, hi = A.n_globals - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (X.node[mid].base_base <= b) lo = mid;
            else hi = mid - 1;
        }
        const TriNode nd = X.node[lo];
        if (nd.nch <= 1) continue;
        int4 *p = (int4 *)X.part + (nd.item_base + (b - nd.base_base) * nd.nch) * tq + wd;
        int4 s = p[0];
        for (int k = 1; k < nd.nch; ++k) {
            const int4 v = p[(int64_t)k * tq];
            s.x += v.x;
            s.y += v.y;
            s.z += v.z;
            s.w += v.w;
        }
        p[0] = s;
    }
}

// Per-lane description of one test of a batch (decoded by the lane that
// evaluates the test's tail).
struct TriTest {
    int64_t item_base;  // the owner's first work item
    int32_t nb, ncg, nch;
    int32_t ru, ry, rz;  // cardinalities: owner, other endpoint, conditioning variable
    int32_t oy, oz;      // one-hot rows of the other endpoint and of z in the owner's tiles
    int32_t e;           // edge record
    uint64_t rank;       // rank of the test in the edge's sequential order
    double alpha, m;
};

// Entry (p, q) of mask cc of the Gram matrices of a node (chunk sums).
BNS_INLINE uint32_t tri_at(const int32_t *part, int64_t item_base, int nb, int ncg, int nch, int cc, int p, int q) {
    if (p > q) {
        const int t = p;
        p = q;
        q = t;
    }
    const int tp = p / kTriT, tq = q / kTriT;
    const int64_t tile = (int64_t)tp * nb - (int64_t)tp * (tp - 1) / 2 + (tq - tp);
    const int64_t item = item_base + (tile * ncg + cc / kTriCats) * nch;
    return (uint32_t)part[item * kTriSlab + (int64_t)(cc % kTriCats) * kTriT * kTriT +
                          (int64_t)(p - tp * kTriT) * kTriT + (q - tq * kTriT)];
}

// Makes a wave's LDS writes visible to its other lanes.
BNS_INLINE void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(kWG) void k_tri_eval(DepthArgs A) {
    constexpr int kCells = kTriMaxCard * kTriMaxCard * kTriMaxCard;
    Ctl *c = A.ctl;
    // per wave: the current test's table N[c][a][b] (index (b ry + a) ru + c),
    // N_u+z[c][b] (b ru + c), N_+yz[a][b] (b ry + a) and N_++z[b]
    __shared__ uint32_t s_tab[kWaves][kCells];
    __shared__ uint32_t s_uz[kWaves][kTriMaxCard * kTriMaxCard];
    __shared__ uint32_t s_yz[kWaves][kTriMaxCard * kTriMaxCard];
    __shared__ uint32_t s_z[kWaves][kTriMaxCard];
    __shared__ int quit;
    __shared__ unsigned long long ntests_sh;
    if (threadIdx.x == 0) {
        quit = (c->done || c->gram_depth != c->depth) ? 1 : 0;
        ntests_sh = c->tri_tests;
    }
    __syncthreads();
    if (quit) return;
    const TriArgs &X = A.tri;
    const unsigned long long ntests = ntests_sh;
    const int lane = threadIdx.x & 63;
    const int wl = (int)(threadIdx.x >> 6);
    const int64_t wave = (int64_t)blockIdx.x * kWaves + wl;
    const int64_t nwaves = (int64_t)gridDim.x * kWaves;
    uint32_t *tab = s_tab[wl];
    uint32_t *uz = s_uz[wl];
    uint32_t *yz = s_yz[wl];
    uint32_t *zz = s_z[wl];
    const int stat_kind = A.tile.stat;
    const bool adjusted = A.tile.df_rule != 0;
    unsigned long long ex = 0;
    double ob = 0.0;
    for (int64_t tb = wave * 64; tb < (int64_t)ntests; tb += nwaves * 64) {
        // lane j decodes test tb + j
        TriTest me;
        me.e = -1;
        const int64_t t = tb + lane;
        if (t < (int64_t)ntests) {
            int lo = 0, hi = A.n_globals - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (X.node[mid].test_base <= t) lo = mid;
                else hi = mid - 1;
            }
            const int g = lo;
            const TriNode nd = X.node[g];
            const ProbDev &P = A.probs[A.var2prob[g]];
            const int u = g - P.var_off;
            const int dm = nd.deg - 1;
            const int tt = (int)(t - nd.test_base);
            // edge (u, k_y-th neighbour) conditioned on the k_z-th neighbour,
            // rank k_z' among the neighbours other than y
            const int ky = tt / dm;
            const int kzp = tt - ky * dm;
            const int kz = kzp + (kzp >= ky ? 1 : 0);
            const int64_t rowb = P.adj_off + (int64_t)u * P.n;
            const int e = X.eidx[rowb + ky];
            if (e >= 0) {
                const int32_t ri = A.edges[e].i;
                const uint64_t nAe = A.edges[e].nA;
                me.item_base = nd.item_base;
                me.nb = nd.nb;
                me.ncg = nd.ncg;
                me.nch = nd.nch;
                me.ru = A.cards[g];
                me.ry = A.cards[P.var_off + A.nbr[rowb + ky]];
                me.rz = A.cards[P.var_off + A.nbr[rowb + kz]];
                me.oy = X.rowoff[rowb + ky];
                me.oz = X.rowoff[rowb + kz];
                me.e = e;
                me.rank = (ri == u ? 0ull : nAe) + (uint64_t)kzp;
                me.alpha = P.alpha;
                me.m = (double)P.m;
            }
        }
        double my_stat = 0.0;
        int64_t my_df = 0;
        // the wave evaluates the batch's tests one after another
        uint64_t todo = __ballot(me.e >= 0);
        while (todo) {
            const int j = __ffsll((long long)todo) - 1;
            todo &= todo - 1;
            const int64_t ib = (int64_t)__shfl((long long)me.item_base, j, 64);
            const int nb = __shfl(me.nb, j, 64), ncg = __shfl(me.ncg, j, 64), nch = __shfl(me.nch, j, 64);
            const int ru = __shfl(me.ru, j, 64), ry = __shfl(me.ry, j, 64), rz = __shfl(me.rz, j, 64);
            const int oy = __shfl(me.oy, j, 64), oz = __shfl(me.oz, j, 64);
            const int ncell = ru * ry * rz;
            for (int i = lane; i < ncell; i += 64) {
                const int cc = i % ru, ab = i / ru, a = ab % ry, b = ab / ry;
                tab[i] = tri_at(X.part, ib, nb, ncg, nch, cc, oy + a, oz + b);
            }
            for (int i = lane; i < ru * rz; i += 64) {
                const int cc = i % ru, b = i / ru;
                uz[i] = tri_at(X.part, ib, nb, ncg, nch, cc, oz + b, oz + b);
            }
            wave_lds_sync();
            for (int i = lane; i < ry * rz; i += 64) {
                uint32_t sacc = 0;
                for (int cc = 0; cc < ru; ++cc) sacc += tab[i * ru + cc];
                yz[i] = sacc;
            }
            if (lane < rz) {
                uint32_t sacc = 0;
                for (int cc = 0; cc < ru; ++cc) sacc += uz[lane * ru + cc];
                zz[lane] = sacc;
            }
            wave_lds_sync();
            double part = 0.0;
            for (int i = lane; i < ncell; i += 64) {
                const int cc = i % ru, ab = i / ru, b = ab / ry;
                const uint32_t nz = zz[b];
                if (nz == 0) continue;
                part += stat_kind ? x2_term<double>(tab[i], uz[b * ru + cc], yz[ab], nz)
                                  : g2_half_term<double>(tab[i], uz[b * ru + cc], yz[ab], nz);
            }
            double dfp = 0.0;
            if (adjusted && lane < rz && zz[lane] > 0) {
                int nrow = 0, ncol = 0;
                for (int cc = 0; cc < ru; ++cc) nrow += uz[lane * ru + cc] > 0u ? 1 : 0;
                for (int a = 0; a < ry; ++a) ncol += yz[lane * ry + a] > 0u ? 1 : 0;
                dfp = (double)(nrow - 1) * (double)(ncol - 1);
            }
            const double st = wave_sum(part);
            const double dfa = adjusted ? wave_sum(dfp) : 0.0;
            if (lane == j) {
                my_stat = stat_kind ? st : 2.0 * st;
                my_df = adjusted ? (int64_t)dfa : (int64_t)(ru - 1) * (int64_t)(ry - 1) * (int64_t)rz;
            }
            wave_lds_sync();  // the tables are rewritten by the next test
        }
        if (me.e >= 0) {
            if (chi2_tail_lane(my_df, my_stat) > me.alpha) atomicMin(&A.min_accept[me.e], (unsigned long long)me.rank);
            ++ex;
            ob += 3.0 * me.m;
            if (A.per_prob) atomicAdd(&A.ecnt[2 * (int64_t)me.e], 1u);
        }
    }
    ex = wave_sum(ex);
    ob = wave_sum(ob);
    if (lane == 0) {
        if (ex) atomicAdd(&c->stats[1].executed, ex);
        if (ob > 0.0) atomicAdd(&c->stats[1].operand_bytes, ob);
        atomicMax(&c->stats[1].t_end, (unsigned long long)wall_clock64());
    }
}

int tri_max_wg_per_cu() {
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tri_gram, kGramWG, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_depth1_gram(const DepthArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_tri_plan, dim3(1), dim3(kPlanThreads), 0, s, a);
    hipLaunchKernelGGL(k_tri_gram, dim3(std::max(1, a.tri.grid)), dim3(kGramWG), 0, s, a);
    hipLaunchKernelGGL(k_tri_reduce, dim3(1024), dim3(kWG), 0, s, a);
    const int eval_grid = std::max(1, a.tri.grid);
    hipLaunchKernelGGL(k_tri_eval, dim3(eval_grid), dim3(kWG), 0, s, a);
    return hipGetLastError();
}

}  // namespace bns
