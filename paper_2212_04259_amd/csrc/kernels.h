// Host-side launchers of the gfx950 kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bns_internal.h"

namespace bns {

// Depth 0 as one contraction (Section IV-B: depth 0 tests every pair with no
// conditioning set).  With one-hot columns A[s][(v, x)] = [X_v(s) = x], every
// pairwise table is a block of the Gram matrix A^T A: N_ij[x][y] =
// (A^T A)[(i, x)][(j, y)], and the diagonal holds each category's count.
// The Gram matrix of each problem is computed in T x T tiles (upper triangle
// of tile blocks) over chunks of samples; each (tile, chunk) work item writes
// its partial tile, and the pair kernel sums a pair's block over the chunks.
struct GramProb {
    const uint8_t *data;   // column v at data + v * ld
    int64_t ld;
    int64_t m;
    int32_t R;             // one-hot columns, padded to a multiple of T
    int32_t nb;            // tile blocks per side (R / T)
    int32_t oh_base;       // first entry of the problem in oh_var / oh_cat
    int32_t nchunks;       // sample chunks of the problem
    int64_t item_base;     // first work item of the problem
    int64_t tile_base;     // first tile of the problem in the summed tiles
};

struct PairArgs {
    const GramProb *gp;    // per problem
    const int32_t *oh_var; // one-hot column -> variable of the problem (-1: padding column)
    const uint16_t *oh_cat; // category of the column (low byte); bit 8: the variable has more than 8 categories
    const int32_t *var_oh; // global variable -> its first one-hot column within its problem
    int32_t *part;         // partial tiles, T * T int32 per work item (null: depth 0 uses the test kernel)
    int32_t *gram;         // tiles summed over the chunks, T * T int32 per tile (= part when no problem has two chunks)
    int64_t items;         // work items over all problems
    int64_t tiles;         // tiles over all problems
    int64_t chunk;         // samples per chunk (a multiple of 64)
    int32_t T;             // tile side: 64 or 128
    int32_t n_gp;
    int32_t gram_grid;     // workgroups of the tile kernel
    int32_t pad;
};

// Depth 1 as masked Gram contractions.  Every depth-1 test of an edge (x, y)
// conditions on one z from the frozen neighbours of one endpoint, the owner u
// of that side (x on side A, y on side B).  With H the one-hot columns of
// u's neighbours and m_c the samples where X_u = c, the masked Gram matrix
// G_c = H^T diag(m_c) H holds N[u = c][v = a][w = b] for every pair of
// neighbours v, w of u: every depth-1 table of the tests u owns is a block of
// G_0 .. G_{r_u - 1}, and the diagonals are the (u, v) marginals.  A work item
// is one T x T tile (upper triangle of tile blocks) of up to four masks of one
// node over one chunk of samples.
constexpr int kTriCats = 4;      // masks (categories of the owner) per work item
constexpr int kTriMinCard = 2;   // cardinality range of the path: at most T / 2 + 1 neighbours per
constexpr int kTriMaxCard = 8;   // tile block, one-hot bytes by one byte permute

struct TriNode {
    int64_t item_base;   // first work item of the node
    int64_t base_base;   // first (tile, category group) pair of the node
    int64_t test_base;   // first depth-1 test owned by the node (deg (deg - 1) tests)
    int32_t deg;         // frozen degree at depth 1 (0: no tests owned)
    int32_t R;           // one-hot rows of the node's neighbours
    int32_t nb;          // tile blocks per side
    int32_t ncg;         // category groups of the node (of up to kTriCats)
    int32_t nch;         // sample chunks
    int32_t pad;
};

struct TriArgs {
    TriNode *node;        // per global variable (null: depth 1 uses the test kernel)
    int32_t *rowoff;      // per problem n*n block as nbr: rowoff[u n + k] = first one-hot row of the
                          // k-th neighbour of u; entry deg holds R
    int32_t *eidx;        // per problem n*n block: edge record of (u, k-th neighbour of u), or -1
    int32_t *part;        // kTriCats T*T int32 per work item (chunk 0 holds the sums)
    int64_t part_items;   // capacity of part in work items
    int32_t target_items; // work items aimed for (sample chunks are cut toward it)
    int32_t grid;         // workgroups of the contraction kernel
};

// Arguments of the per-depth pipeline of a skeleton search (all device pointers).
struct DepthArgs {
    const ProbDev *probs;
    int32_t n_probs;
    int32_t n_globals;        // sum of n over problems
    const int32_t *var2prob;  // global variable -> problem
    const uint8_t *cards;     // per global variable
    const uint64_t *binom;    // binom[n * kBinomK + k], saturated
    int32_t binom_rows;
    int32_t pad;
    uint8_t *adj;             // per problem n*n block at adj_off
    int32_t *nbr;             // frozen adjacency lists, same blocks as adj
    int32_t *ipos;            // ipos[v * n + u] = position of u in the frozen list of v
    uint64_t *adjbits;        // small searches: adjacency bit rows, ceil(n / 64) words per row
    int64_t bit_words;        // words of adjbits over all problems
    int32_t *deg;             // per global variable
    int32_t *rowcnt;          // per global variable: alive edges (v, u > v)
    int64_t *rowbase;         // exclusive scan of rowcnt
    EdgeRec *edges_tmp;
    EdgeRec *edges;           // sorted by levels, descending
    unsigned long long *min_accept;
    // Multi-dataset searches (per_prob = 1): per-problem counters, and per
    // edge of the current depth the tests executed and re-checked
    // (ecnt[2 e], ecnt[2 e + 1]), summed by problem at removal time.
    PStatDev *pstat;
    uint32_t *ecnt;
    int32_t per_prob;
    int32_t pad3;
    // Verification mode (err_val non-null): every executed test appends its
    // relative FP32 error and a tag (problem << 16 | flip << 8 | depth).
    float *err_val;
    uint32_t *err_tag;
    unsigned long long *err_cnt;  // entries appended (may exceed err_cap: overflow)
    int64_t err_cap;
    int8_t *rdepth;           // per pair (problem block), removal depth or -1
    int32_t *pool;            // removal records of depth >= 1: problem, i, j, sepset
    Ctl *ctl;
    Tile tile;
    int64_t n_pairs;          // variable pairs over all problems
    int32_t test_waves;       // waves of the persistent test grid
    int32_t edge_grid;        // workgroups of the per-edge kernels (scatter, removal)
    // Sample splitting of depths with few tests: a test's samples are cut
    // into chunks counted by different groups and merged into a per-ticket
    // table in split_tab (all zero between tests); split_cnt[ticket] counts
    // the chunks merged so far (zero between tests).
    uint32_t *split_tab;
    uint32_t *split_cnt;
    int64_t split_words;      // words of split_tab
    int64_t split_tickets;    // entries of split_cnt: depths with more tickets are not split
    int64_t m_max;            // largest sample count over problems
    int32_t split_min;        // smallest chunk in samples; <= 0 disables splitting
    int32_t units_per_group;  // work units aimed for per concurrent group when splitting
    int32_t mode_policy;      // 0 automatic, 1 one test per wave, 2 one test per workgroup
    int32_t grab_fixed;       // tickets per grab (0: from the ticket count)
    int32_t grab_block_log2;  // test kernel: units dealt to a grab counter in runs of 2^this (0 or kGrabRunLog2)
    uint32_t wave_depths;     // depths d < 32 with bit d set: one test per wave (overrides mode_policy)
    uint32_t block_depths;    // same, one test per workgroup
    int32_t round_width;      // ticket levels: 0 doubling (level L: ranks [2^L - 1, 2^(L+1) - 1)); g > 0
                              // rounds of g ranks (level L < 63: [L g, (L + 1) g); level 63: the rest)
    int32_t edge_form;        // 1: one group per edge runs its tests in order to the first accept
    int32_t xy_policy;        // depth 1: a work unit is one edge's ranks of a level, counted in one pass
                              // sharing the X and Y columns (0 never, 1 always)
    int32_t pad2;
    // Results of a launch, written into pinned host memory by its last kernel.
    Ctl *h_ctl;               // copy of the control block
    char *h_res;              // null, or removal depths (res_rbytes) then the first removal records
    int64_t res_rbytes;       // adjacency bytes rounded up to 8 (rdepth holds at least this many)
    int64_t res_pool_words;   // removal-record words copied at most
    // Completion flag: the last workgroup of the publishing kernel, after all
    // copies are visible to the host, writes ++*pub_seq into *h_flag.
    unsigned long long *pub_seq;  // device: launches published so far
    unsigned int *pub_cnt;        // device: workgroups of the current publish done (0 between)
    unsigned long long *h_flag;   // pinned host
    PairArgs pairs;               // depth 0 as one contraction (pairs.part non-null)
    TriArgs tri;                  // depth 1 as masked contractions (tri.node non-null)
};

// Small searches keep the adjacency as bit rows in LDS and prepare each depth
// inside the removal kernel of the depth before.
constexpr int kSmallBitWords = 4096;
constexpr int kGrabRunLog2 = 6;  // runs of 64 tickets per grab counter (large searches)
__host__ __device__ bool small_search(const DepthArgs &a);
hipError_t launch_depth_prepare(const DepthArgs &a, hipStream_t s);   // snapshot .. scatter
// With start/stop events the runtime records them with the kernel's own
// dispatch (tight bracketing of short kernels).
// units: the instance for the depth's work units: 0 one test, 1 (edge, level)
// groups (depth 1 with a.xy_policy), 2 one test of at most kNarrowDepth + 2
// columns (the instance without the wider counting loops, whose registers
// otherwise spill); the host's choice for a depth must match depth_units().
hipError_t launch_depth_tests(const DepthArgs &a, int grid, hipStream_t s,
                              hipEvent_t start = nullptr, hipEvent_t stop = nullptr, int units = 0);
constexpr int kNarrowDepth = 2;
// Work units of depth d (the rule the depth preparation applies).
inline int depth_units(const DepthArgs &a, int d) {
    if (a.edge_form || a.err_val) return 0;
    if (a.xy_policy == 1 && d == 1 && a.round_width == 0) return 1;
    if (d <= kNarrowDepth && a.tile.stat == 0 && a.tile.df_rule == 0) return 2;
    return 0;
}
hipError_t launch_depth_apply(const DepthArgs &a, hipStream_t s);     // removals + finalize
// LDS increment throughput: grid workgroups of kWG lanes, 16 * steps
// increments per lane; sink receives the increments' total.
hipError_t launch_lds_rate(int grid, int steps, unsigned int *sink, hipStream_t s);
hipError_t launch_init_search(const DepthArgs &a, hipStream_t s);     // complete graph, reset
hipError_t launch_publish(const DepthArgs &a, hipStream_t s);         // results into pinned host memory
// Depth 0 through the pair contraction: Gram tiles, then one decision per pair
// (in place of the depth's test kernel).
hipError_t launch_depth0_pairs(const DepthArgs &a, hipStream_t s);
// Every pairwise test of one dataset (pair index i n - i (i + 1) / 2 + j - i - 1).
hipError_t launch_ci_pairs(const PairArgs &p, const uint8_t *cards, int32_t n, double alpha, int stat,
                           int df_rule, double *stat_out, int64_t *df_out, double *p_out, int32_t *flags_out,
                           hipStream_t s);
int gram_max_wg_per_cu(int T);
// Depth 1 through the masked contractions: plan, tiles, chunk sums and one
// decision per test (the depth's test kernel then returns at once).  Runs
// only when the control block's depth is 1; falls back to the test kernel
// when the plan exceeds the tile buffer.
hipError_t launch_depth1_gram(const DepthArgs &a, hipStream_t s);
int tri_max_wg_per_cu();
int depth_tests_max_wg_per_cu(int lds_bytes);
int depth_tests_fit_lds(int lds_per_cu);  // default dynamic LDS at full occupancy
hipError_t allow_dynamic_lds(int bytes);  // raises the per-kernel dynamic LDS limit

// Batched CI tests without PC control: results as records (out) or, with
// out null, as separate arrays (soa).
struct CiOutSoa {
    double *g2;
    double *p;
    int64_t *df;
    int32_t *flags;
};
hipError_t launch_ci_batch(const uint8_t *data, int64_t ld, int64_t m, const uint8_t *cards,
                           const CiTestDev *tests, const int32_t *zpool, int64_t n_tests,
                           double alpha, Tile tile, CiOutDev *out, uint32_t *tables,
                           const int64_t *table_off, int grid, hipStream_t s,
                           CiOutSoa soa = CiOutSoa{nullptr, nullptr, nullptr, nullptr});

// Plain per-test form: sample-parallel count of one test into per-block
// partial tables, then a single-workgroup finish (fixed-order sum, FP64 G^2).
struct PlainTest {
    int32_t vars[kMaxCols];
    int32_t ncols;
    int32_t pad;
};
hipError_t launch_plain_count(const uint8_t *data, int64_t ld, int64_t m, const uint8_t *cards,
                              const PlainTest &t, int64_t samples_per_block, int nblocks,
                              uint32_t *partials, int64_t T, int lds_words, hipStream_t s);
hipError_t launch_plain_finish(const uint8_t *cards, const PlainTest &t, int nblocks,
                               const uint32_t *partials, int64_t T, uint32_t *table_ws,
                               double alpha, int stat, int df_rule, CiOutDev *out, hipStream_t s);

// Checks every value against its cardinality; first offending flat index
// (v * m + s) is atomically minimised into *bad (initialised to INT64_MAX).
hipError_t launch_validate(const uint8_t *data, int64_t ld, int64_t m, int32_t n,
                           const uint8_t *cards, unsigned long long *bad, hipStream_t s);

}  // namespace bns
