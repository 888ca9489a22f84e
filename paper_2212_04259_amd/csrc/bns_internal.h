// Internal types shared by the host driver and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bns {

constexpr int kWG = 256;            // threads per workgroup (4 wave64)
constexpr int kWaves = kWG / 64;
// Largest conditioning set a kernel accepts.  Tables are limited to 2^24
// cells and, from depth 1 on, every conditioning variable has at least two
// categories (a one-category variable fails no test and leaves the graph at
// depth 0), so no admissible test has more than 22 conditioning variables.
constexpr int kMaxZ = 22;
constexpr int kMaxCols = kMaxZ + 2;
constexpr int kBinomK = kMaxZ + 1;  // binomial table columns: k = 0..kMaxZ
constexpr int kMaxLevels = 64;      // ticket levels: level L holds test ranks [2^L - 1, 2^(L+1) - 1)
constexpr uint32_t kMaxCells = 1u << 24;  // largest contingency table (cells)
constexpr int kMaxDepths = 64;      // depth records kept per search
constexpr int kSlotsPerWave = 8;    // tickets decoded per grab, per wave
constexpr int kGrabParts = 8;       // work-unit counters of the test kernel (one per XCD's workgroups)
constexpr int kGrabStride = 16;     // 64-bit words between two counters (one 128-byte line each)
constexpr int kBinomLds = 512;      // binomial entries of a depth staged for the test kernel

// Status codes written by kernels into the control block.
enum DevError : int32_t {
    kDevOk = 0,
    kDevTableTooLarge = 1,
    kDevTooManyTests = 2,
    kDevDepthTooLarge = 3,
    kDevUnitMismatch = 4  // the test kernel instance does not match the depth's work units
};

// One dataset of a (possibly multi-dataset) skeleton search.
struct ProbDev {
    const uint8_t *data;  // column v at data + v * ld
    int64_t ld;
    int64_t m;
    int32_t n;
    int32_t var_off;      // first global variable index (cards, degree, neighbour rows)
    int64_t adj_off;      // offset of this problem's n*n block in adjacency / pair arrays
    double alpha;
    int32_t max_depth;    // -1: unbounded
    int32_t bit_off;      // first word of this problem's adjacency bit rows (small searches)
};

// One surviving edge (i < j, local ids) at the current depth.
struct EdgeRec {
    int32_t prob;
    int32_t i, j;
    int32_t posj;         // position of j in the frozen list a(i)
    int32_t posi;         // position of i in a(j)
    int32_t levels;       // number of ticket levels the edge takes part in
    int32_t pA;           // |a(i)\{j}|
    int32_t pB;           // |a(j)\{i}|
    uint64_t nA;          // tests on side A (subsets of a(i)\{j})
    uint64_t n;           // all tests of the edge
};

// Per-depth counters kept on the device.
struct DepthStatDev {
    unsigned long long edges;
    unsigned long long required;
    unsigned long long executed;
    unsigned long long removed;
    unsigned long long rechecks;
    unsigned long long tickets;
    double operand_bytes;
    unsigned long long t_start;      // entry of the test kernel's workgroup 0, 100 MHz device clock
    unsigned long long t_end;        // latest workgroup end
    int32_t mode;                    // 0 one test per wave, 1 per workgroup
    int32_t chunks;                  // sample chunks per test (1: not split)
    long long chunk_len;             // samples per chunk
};

// Per-problem, per-depth counters of a multi-dataset search (problem k,
// depth d at index k * kMaxDepths + d).
struct PStatDev {
    unsigned long long edges;     // edges of the problem alive when the depth started
    unsigned long long tickets;   // tests of the depth's sequential order (all ranks)
    unsigned long long required;  // canonical tests: per edge, up to its first accepting one
    unsigned long long removed;
    unsigned long long executed;  // tests run (speculative included)
    unsigned long long rechecks;
};

// Device-resident control block of a skeleton search.
struct Ctl {
    int32_t depth;         // depth being built / run
    int32_t done;          // 1 once a depth has no tests (search finished)
    int32_t error;         // DevError
    int32_t pad0;
    unsigned long long n_edges;        // edges in the current list
    unsigned long long total_tickets;
    unsigned long long pool_used;      // sepset members written so far
    unsigned int apply_done;           // blocks of the removal kernel that finished
    int32_t maxdeg;                    // largest frozen adjacency set at this depth
    unsigned long long maxn;           // most tests of one edge at this depth (fixed-width levels)
    int32_t mode;                      // test kernel: 0 one test per wave, 1 per workgroup
    int32_t batch;                     // work units taken per grab
    int32_t chunks;                    // sample chunks per test (1: tests are not split)
    unsigned long long total_units;    // total_tickets * chunks
    long long chunk_len;               // samples per chunk (a multiple of 1024)
    unsigned long long split_cap;      // cells of each ticket's merge table
    // Depth 1 through the masked Gram contractions: the depth whose tests
    // the contraction ran (-1: none), its work items, (tile, category group)
    // pairs, the longest chunk count of a node and the samples per chunk.
    int32_t gram_depth;
    int32_t tri_nch_max;
    int32_t xy;                        // test kernel units: 0 tests, 1 (edge, level) groups
    int32_t pad1;
    unsigned long long tri_items;
    unsigned long long tri_base;
    unsigned long long tri_tests;
    long long tri_chunk;
    unsigned long long level_base[kMaxLevels + 1];
    unsigned long long level_cnt[kMaxLevels + 1];
    unsigned int hist[kMaxLevels + 2];
    unsigned int cursor[kMaxLevels + 2];
    // Binomials C(n, k), n <= maxdeg, k <= depth, row stride depth + 1, for
    // the test kernel's unranking (bstride 0: not staged, use the full table).
    int32_t bstride, brows;
    uint64_t bslice[kBinomLds];
    DepthStatDev stats[kMaxDepths];
    // Work-unit counters of the test kernel: after every group's first batch
    // (taken without a counter), unit S0 + p + kGrabParts * i is the i-th of
    // counter p.  One line each: same-address atomics serialise.
    alignas(128) unsigned long long grab_ctr[kGrabParts * kGrabStride];
};

// One CI test for the batch entry point.
struct CiTestDev {
    int32_t x, y, nz, zoff;
};

struct CiOutDev {
    double g2;
    double p;
    int64_t df;
    int32_t flags;
    int32_t pad;
};

// Tunables of a launch.
struct Tile {
    int32_t lds_words;     // dynamic LDS per workgroup, in 32-bit words
    int32_t max_rep_log2;  // cap on per-table replication (log2)
    int32_t fp64;          // 1: FP64 statistic; 0: FP32 + FP64 recheck
    int16_t stat;          // 0: G^2; 1: Pearson X^2
    int16_t df_rule;       // 0: df from the declared cards; 1: adjusted for empty rows, columns, strata
    double band;           // recheck band on |p - alpha|
};

}  // namespace bns
