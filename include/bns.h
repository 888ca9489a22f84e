/*
 * bns.h -- C ABI of the MI355X (gfx950) batched G^2 conditional-independence
 * engine for PC-stable skeleton learning.
 *
 * Method: Jiang, Wen, Mian, "Fast Parallel Bayesian Network Structure
 * Learning".  The library runs step 1 of PC-stable (Section III-C,
 * Algorithm 1): starting from the complete undirected graph, at depth
 * d = 0, 1, 2, ... every surviving edge (V_i, V_j) is tested for conditional
 * independence given every size-d subset S of the frozen adjacency sets
 * a(V_i)\{V_j}, then a(V_j)\{V_i} (the grouping of Section IV-C), in
 * lexicographic order (Section IV-C), until one test accepts; the edge is then
 * removed and S is its separating set.  Depth 0 runs one marginal test per
 * pair (Section IV-B).  Each test is the G^2 test of Section III-B.
 *
 * Conventions shared by every entry point
 *   - Data layout: variable-major ("transposed") uint8 columns, as in the
 *     cache-friendly storage of Section IV-C: value of variable v in sample s
 *     at data[v * ld + s], with ld = n_samples for host buffers.  Values must
 *     lie in [0, cards[v]); cards[v] in [1, 255].
 *   - Contingency table cell of (x, y, z_1..z_d):
 *       cell = x + r_X * (y + r_Y * zc),  zc = sum_k z_k * prod_{l<k} r_{z_l}
 *     (first conditioning variable fastest).
 *   - G^2 = 2 sum_{xyz} N_xyz ln(N_xyz / E_xyz), E_xyz = N_x+z N_+yz / N_++z,
 *     cells with N_xyz = 0 contribute 0 (Section III-B; natural log).
 *   - df = (r_X - 1)(r_Y - 1) prod_k r_{z_k}, from the declared cards, with no
 *     adjustment for empty cells (Section III-B gives the first two factors;
 *     the conditioning factor is the standard one for a stratified test).
 *   - p = Q(df / 2, G^2 / 2), the chi-square upper tail, always in FP64;
 *     df = 0 gives p = 1.  Independence is declared iff p > alpha (strict).
 *   - Sepset choice: among the tests of an edge in the order above, the first
 *     accepting one; parallel forms reproduce exactly this choice.
 *   - Counts are exact (int32 per cell; n_samples < 2^31).
 *   - Errors: every entry point returns a bns_status; on failure nothing is
 *     written to caller outputs beyond what the function documents, and
 *     bns_last_error() describes the failure.  No exception crosses the ABI.
 *   - Ownership: input buffers are borrowed for the duration of the call.
 *     Handles (bns_dataset, bns_skeleton) are owned by the library until the
 *     matching *_free.  Output arrays are allocated by the caller.
 *   - Device and streams: work runs on the HIP device that is current on the
 *     calling thread when the dataset is created; opt->stream selects the HIP
 *     stream (NULL = the device's default stream).  Calls on one device are
 *     serialised by the library; handles are not thread-safe.
 */
#ifndef BNS_H
#define BNS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BNS_VERSION 2

typedef enum bns_status {
    BNS_OK = 0,
    BNS_E_INVALID_ARG = 1,      /* NULL pointer, bad size, alpha not in (0,1), ... */
    BNS_E_VALUE_RANGE = 2,      /* a data value >= its variable's cardinality */
    BNS_E_TABLE_TOO_LARGE = 3,  /* a test's table exceeds the supported cell count */
    BNS_E_NOMEM = 4,            /* device or host allocation failed */
    BNS_E_DEVICE = 5,           /* no usable device, or a HIP call failed */
    BNS_E_INTERNAL = 6
} bns_status;

/* Execution form of the skeleton search. */
enum {
    BNS_FORM_BATCHED = 0, /* device-resident per-depth work queue, one persistent launch per depth */
    BNS_FORM_PLAIN = 1,   /* host walks the tests in order; one sample-parallel launch per test */
    BNS_FORM_EDGE = 2     /* one persistent launch per depth in which each group of lanes (a wave,
                             or a workgroup with test_group 2) takes one edge at a time and runs
                             its tests in order until the first accepting one (the edge-level
                             parallelism of Section IV-A: no speculative test) */
};

/* Arithmetic of the G^2 log-sum (counts are always exact integers and the
 * p-value is always FP64). */
enum {
    BNS_PREC_FP32_RECHECK = 0, /* FP32 G^2; FP64 re-evaluation near alpha */
    BNS_PREC_FP64 = 1          /* FP64 G^2 */
};

typedef struct bns_options {
    int32_t form;          /* BNS_FORM_*; default BATCHED */
    int32_t precision;     /* BNS_PREC_*; default FP32_RECHECK */
    double recheck_band;   /* FP32 mode: decisions with |p - alpha| < band (or within the
                              propagated FP32 error bound) are re-evaluated in FP64;
                              default 1e-3 */
    int32_t lds_bytes;     /* LDS budget per workgroup for tables; 0 = default */
    int32_t wg_per_cu;     /* persistent-grid workgroups per compute unit; 0 = default */
    int32_t use_graph;     /* batched form: replay the per-depth launch sequence as a
                              hipGraph; default 1 */
    int32_t timing;        /* record HIP events around each depth's test launch; the
                              durations appear in bns_depth_stats.kernel_seconds */
    int32_t split_min_samples; /* batched form: a depth with too few tests to occupy the
                              device cuts each test's samples into chunks of at least this
                              many samples, counted by different groups of lanes and merged
                              exactly (integer counts) before G^2; 0 = default (4096),
                              -1 = never split */
    int32_t units_per_group;   /* batched form: a depth is split only when it has at least
                              two chunks per test for every units_per_group groups of
                              lanes; 0 = default (1) */
    int32_t test_group;    /* batched form: lanes that run one test: 0 = automatic,
                              1 = one wave (64 lanes), 2 = one workgroup (256 lanes) */
    int32_t max_replicas;  /* copies of a contingency table in LDS that lanes increment
                              (summed before G^2); a power of two in [1, 64]; 0 = default */
    int32_t tickets_per_grab; /* batched form: tests a group takes per grab of a ticket
                              counter, in [1, 8]; 0 = automatic */
    int32_t ticket_runs;   /* batched form: tickets dealt to the test kernel's grab
                              counters one at a time (1) or in runs of 64 consecutive
                              tickets (2: edges that share a column run on one XCD);
                              0 = automatic (runs when the search's columns exceed
                              64 MiB) */
    uint32_t wave_depths;  /* batched form: per-depth override of test_group for depths
                              d < 32: bit (1u << d) set = one wave per test at depth d */
    uint32_t block_depths; /* same, one workgroup per test; no bit may be set in both */
    int32_t report_errors; /* batched form, FP32 arithmetic: verification mode (untimed use).
                              Every executed test is also evaluated in FP64 (from the
                              table still in LDS, or by counting again) and the relative
                              FP32 G^2 error |G2_32 - G2_64| / max(G2_64, 1) and the
                              decisions the FP32 value alone would have flipped are
                              reported per depth in bns_depth_stats (err_* fields).
                              Decisions, skeleton and sepsets are those of the normal
                              search.  0 = off (default) */
    int32_t workspace_mb;  /* largest device workspace a call may hold, in MiB (datasets
                              excluded); a call that needs more fails with BNS_E_NOMEM
                              before any device work.  0 = no limit (default) */
    int32_t statistic;     /* BNS_STAT_*: the test statistic (default BNS_STAT_G2) */
    int32_t df_rule;       /* BNS_DF_*: the degrees of freedom (default BNS_DF_DECLARED) */
    int32_t depth0;        /* batched form, depth 0 (one marginal test per pair):
                              BNS_DEPTH0_* (default automatic) */
    int32_t round_tests;   /* batched form: ranks of an edge per level of the depth's work queue
                              (the counterpart of the group size gs of Section IV-B).  The
                              queue holds level after level, each giving every edge that still
                              has tests its next ranks: 0 = levels of 1, 1, 2, 4, 8, ... ranks
                              (default); g in [1, 65536] = levels of g ranks (the last of 64
                              levels takes the rest).  A test whose edge has accepted at a
                              lower rank is skipped when it is taken; those run before the
                              accept was seen count as executed (speculative) tests */
    int32_t depth1;        /* batched form, depth 1 (conditioning sets of one variable):
                              BNS_DEPTH1_* (default automatic) */
    int32_t group_tests;   /* batched form, depth 1 in the test kernel: BNS_GROUP_* (default
                              automatic) */
    void *stream;          /* hipStream_t; NULL = default stream */
} bns_options;

/* Test statistic (Section III-B defines G^2; Section II names Pearson's X^2 as
 * an alternative test on the same contingency table).  Both are compared with
 * the chi-square distribution of the same df. */
enum {
    BNS_STAT_G2 = 0, /* G^2 = 2 sum N ln(N / E) (the paper's test) */
    BNS_STAT_X2 = 1  /* X^2 = sum (N - E)^2 / E over cells with E > 0 */
};

/* Degrees of freedom of a test. */
enum {
    BNS_DF_DECLARED = 0, /* (r_X - 1)(r_Y - 1) prod r_Z from the declared cardinalities */
    BNS_DF_ADJUSTED = 1  /* sum over strata z with N_++z > 0 of (a_z - 1)(b_z - 1), where a_z
                            and b_z count the non-empty rows N_x+z and columns N_+yz of the
                            stratum (empty categories and strata dropped); df 0 gives p = 1 */
};

/* Depth-0 path of the batched form. */
enum {
    BNS_DEPTH0_AUTO = 0,    /* PAIRS when the depth's pair-samples (pairs times samples, summed
                               over the problems) reach 5e8 and the partial tiles fit, else TESTS */
    BNS_DEPTH0_TESTS = 1,   /* the depth's tests run in the per-depth test kernel */
    BNS_DEPTH0_PAIRS = 2    /* all pairwise tables at once as one contraction of one-hot
                               columns (Section IV-B: depth 0 tests every pair); the
                               statistic is evaluated in FP64.  Verification mode
                               (report_errors) keeps depth 0 in the test kernel */
};

/* Depth-1 path of the batched form. */
enum {
    BNS_DEPTH1_AUTO = 0,    /* TESTS (the contraction evaluates every depth-1 test, where the
                               sequential order stops an edge at its first accepting test:
                               measured slower on all five benchmark workloads) */
    BNS_DEPTH1_TESTS = 1,   /* the depth's tests run in the per-depth test kernel */
    BNS_DEPTH1_GRAM = 2     /* every depth-1 table as a block of masked Gram matrices: for
                               each node u and category c of u, the one-hot columns of u's
                               frozen neighbours multiplied over the samples with X_u = c
                               (int8 MFMA, exact counts); every depth-1 test is evaluated,
                               in FP64, and each edge keeps its first accepting test, so the
                               results are those of Algorithm 1.  Needs cardinalities in [2, 8];
                               otherwise, in verification mode, in the edge-level form, or
                               when the plan exceeds the tile buffer, the test kernel runs */
};

/* Work units of depth 1 in the test kernel (the counterpart of Section IV-B's
 * group of tests of one edge). */
enum {
    BNS_GROUP_AUTO = 0,   /* EDGE when the search's columns (variables x samples bytes of
                             all its datasets) exceed 64 MiB, a quarter of MI355X's last-level
                             cache (its tests would re-read X and Y from DRAM), else TEST */
    BNS_GROUP_TEST = 1,   /* one test per work unit */
    BNS_GROUP_EDGE = 2    /* one edge's ranks of a work-queue level per unit, counted in one
                             pass over the samples that loads X and Y once and adds each
                             test's table (up to 8 per pass; the unit stops after the pass
                             with its first acceptance).  Doubling levels only (round_tests
                             0); verification mode keeps one test per unit */
};

/* Fills *opt with the defaults.  opt must not be NULL. */
void bns_options_default(bns_options *opt);

/* Human-readable description of the last failure on the calling thread; valid
 * until the next call into the library on this thread.  Never NULL. */
const char *bns_last_error(void);

/* ---------------------------------------------------------------------- */
/* Datasets resident in device memory                                     */
/* ---------------------------------------------------------------------- */
typedef struct bns_dataset bns_dataset;

/* Copies host data (uint8 [n_vars][n_samples], row v = variable v) and cards
 * (uint8 [n_vars]) to the current device.  Every value is checked against its
 * cardinality; the first offending (variable, sample) is reported as
 * BNS_E_VALUE_RANGE.  n_samples in [1, 2^31 - 1], n_vars in [2, 65535]. */
bns_status bns_dataset_create(const uint8_t *data, int64_t n_samples, int32_t n_vars,
                              const uint8_t *cards, bns_dataset **out);

/* Wraps device memory owned by the caller (e.g. a torch tensor): value of
 * variable v in sample s at d_data[v * ld + s].  d_data must be 16-byte aligned
 * and ld a multiple of 16 with ld >= n_samples; the memory must outlive the
 * handle.  cards is a host array.  Values are checked on the device. */
bns_status bns_dataset_wrap_device(const uint8_t *d_data, int64_t ld, int64_t n_samples,
                                   int32_t n_vars, const uint8_t *cards, bns_dataset **out);

void bns_dataset_free(bns_dataset *ds);

/* ---------------------------------------------------------------------- */
/* Batched CI tests (no PC control)                                       */
/* ---------------------------------------------------------------------- */

/* One test I(x, y | z): the conditioning variables are
 * z_pool[z_offset .. z_offset + n_z). */
typedef struct bns_ci_test {
    int32_t x, y, n_z, z_offset;
} bns_ci_test;

/* Result flag bits of bns_ci_batch. */
enum {
    BNS_CI_INDEPENDENT = 1, /* p > alpha */
    BNS_CI_RECHECKED = 2    /* FP32 mode: decided by the FP64 re-evaluation */
};

/* Runs n_tests G^2 tests on ds as given (Section III-B), in the precision of
 * opt->precision.  All pointers are host pointers; outputs have n_tests
 * entries: g2 (the statistic the decision used: FP64 when rechecked or in FP64
 * mode), df, p, flags.  Any output may be NULL.  tables_out, when not NULL,
 * receives each test's exact counts at tables_out[table_offsets[t] ..
 * + r_x r_y prod r_z) in the cell layout above (table_offsets must then be
 * given).  Tests must have x != y, z disjoint from {x, y}, ids in range;
 * violations give BNS_E_INVALID_ARG before any device work. */
bns_status bns_ci_batch(const bns_dataset *ds, const bns_ci_test *tests, int64_t n_tests,
                        const int32_t *z_pool, int64_t z_pool_len, double alpha,
                        const bns_options *opt, double *g2, int64_t *df, double *p,
                        int32_t *flags, int32_t *tables_out, const int64_t *table_offsets);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): bns_ci_batch without any
 * allocation by the library.  The tests, the conditioning pool and the results
 * are staged in a fixed device scratch area of BNS_NOALLOC_SCRATCH_BYTES that
 * the library holds on each device it runs on until the process ends, instead
 * of library-allocated buffers; no hipMalloc, hipFree or pinned host
 * allocation happens in the call.  Same arguments, checks, kernels and results
 * as bns_ci_batch (all pointers are host pointers; outputs may be NULL), minus
 * the table output.  A call needs 16 n_tests + 4 z_pool_len + 28 n_tests bytes
 * of scratch (each section rounded up to 256 bytes); a larger one fails with
 * BNS_E_NOMEM before any device work.  Calls are synchronous (the stream of
 * opt->stream, NULL = the null stream, is synchronised before returning) and
 * the library serialises calls per device, so they never overlap on a device
 * within a process; overlapping calls would race on the shared scratch area,
 * which keeps the last call's contents.  The dataset must have been created
 * beforehand (that allocates). */
#define BNS_NOALLOC_SCRATCH_BYTES (16 << 20)
bns_status bns_ci_batch_noalloc(const bns_dataset *ds, const bns_ci_test *tests, int64_t n_tests,
                                const int32_t *z_pool, int64_t z_pool_len, double alpha,
                                const bns_options *opt, double *g2, int64_t *df, double *p,
                                int32_t *flags);

/* Every pairwise marginal test of ds at once: the tests of depth 0 of the
 * skeleton search (Section IV-B: one test per pair, no conditioning set), all
 * n(n-1)/2 tables formed together as blocks of the Gram matrix of one-hot
 * columns (an int8 matrix-core contraction; exact integer counts).  Pair
 * (i, j), i < j, is entry i n - i (i + 1) / 2 + j - i - 1 of each output
 * (host arrays of n(n-1)/2 entries, any may be NULL): the statistic
 * (opt->statistic, evaluated in FP64), df (opt->df_rule), p (FP64) and flags
 * (BNS_CI_INDEPENDENT when p > alpha). */
bns_status bns_ci_pairs(const bns_dataset *ds, double alpha, const bns_options *opt, double *stat,
                        int64_t *df, double *p, int32_t *flags);

/* ---------------------------------------------------------------------- */
/* PC-stable skeleton (Algorithm 1)                                       */
/* ---------------------------------------------------------------------- */
typedef struct bns_skeleton bns_skeleton;

/* Per-depth counters of a skeleton search. */
typedef struct bns_depth_stats {
    int32_t depth;
    int32_t test_group;      /* batched form: lanes per test at this depth, 1 = one wave,
                                2 = one workgroup, 3 = depth 0 ran as the pair contraction
                                (bns_ci_pairs' tables); 0 in the plain form */
    int64_t edges;           /* edges alive when the depth started */
    int64_t tests_required;  /* tests in the canonical sequential order: per edge, up to
                                and including its first accepting test */
    int64_t tests_executed;  /* tests run, including speculative ones */
    int64_t removed;         /* edges removed at this depth */
    int64_t rechecks;        /* FP32 decisions re-evaluated in FP64 */
    int64_t tickets;         /* work items scheduled (batched form) */
    double operand_bytes;    /* sum over executed tests of (d + 2) * n_samples */
    double kernel_seconds;   /* test-launch time from HIP events around the launch
                                (opt->timing; includes the dispatch gap), else 0 */
    double span_seconds;     /* test-kernel execution span from device clock stamps:
                                entry of workgroup 0 (dispatched first) to the end of
                                the last workgroup (always) */
    /* Verification mode (options.report_errors), else 0: */
    int64_t err_tests;       /* executed tests whose FP32 statistic was compared with FP64 */
    int64_t err_flips;       /* of those, tests whose FP32-only decision differs from FP64's
                                (the re-check band exists to catch these) */
    double err_max;          /* largest relative FP32 error of the statistic */
    double err_p50;          /* median */
    double err_p99;          /* 99th percentile */
    /* Samples per work unit at this depth (0 in the plain form): */
    int32_t chunks;          /* sample chunks each test was cut into (1: not split; 0 for
                                the pair contraction) */
    int32_t reserved;
    int64_t chunk_samples;   /* samples per chunk (the longest dataset's count when not
                                split; the pair contraction's sample chunk) */
} bns_depth_stats;

/* Learns the skeleton of one dataset.  alpha in (0, 1); max_depth >= -1
 * (depths 0..max_depth; -1 = until no edge has a conditioning set of size d).
 * Host data as in bns_dataset_create. */
bns_status bns_pc_skeleton(const uint8_t *data, int64_t n_samples, int32_t n_vars,
                           const uint8_t *cards, double alpha, int32_t max_depth,
                           const bns_options *opt, bns_skeleton **out);

/* Same, on a dataset already resident on the device. */
bns_status bns_pc_skeleton_dataset(const bns_dataset *ds, double alpha, int32_t max_depth,
                                   const bns_options *opt, bns_skeleton **out);

/* Learns the skeletons of n_problems independent datasets together, one
 * launch per depth covering all of them (batched form only).  alpha and
 * max_depth are per problem; outs receives n_problems handles. */
bns_status bns_pc_skeleton_batch(const bns_dataset *const *ds, int32_t n_problems,
                                 const double *alpha, const int32_t *max_depth,
                                 const bns_options *opt, bns_skeleton **outs);

/* Chooses launch options for the batched search of these datasets by timing
 * complete trial searches, each candidate measured `trials` times (median;
 * 0 = 5).  Searched, each only where base leaves it open (0 / AUTO):
 *   1. lanes per test, per depth (wave_depths / block_depths), from the depth
 *      spans of trial searches with one wave and one workgroup per test;
 *   2. every combination of replication cap, LDS budget and tests per grab
 *      (a grid of at most 27), then step 1 again under the chosen options;
 *   3. samples per work unit: split_min_samples in {default, 2048, 8192,
 *      16384, never} x units_per_group in {default, 4, 16};
 *   4. depth 1's work units (one test, or one edge's ranks of a level) and
 *      its path (the test kernel or the masked contractions);
 *   5. the depth-0 path (the test kernel or the pair contraction);
 *   6. tests per grab again, then step 1 again, under the paths of 4 and 5.
 * A candidate is kept only if the whole search gets clearly faster.  *best
 * receives base with the chosen options filled in (base NULL = defaults).
 * The choice is cached per device (architecture and compute units) and
 * workload (problem sizes, alphas, max depths, precision, statistic, the
 * options base fixes): in memory, and appended to a text file that later
 * processes read: $BNS_TUNE_CACHE if set, else $XDG_CACHE_HOME/bns_autotune.txt,
 * else $HOME/.cache/bns_autotune.txt; a file that cannot be read or written
 * is skipped silently (options never change results).  Repeated calls for a
 * cached workload return at once.  The trial searches run on the device like
 * bns_pc_skeleton_batch. */
bns_status bns_autotune(const bns_dataset *const *ds, int32_t n_problems, const double *alpha,
                        const int32_t *max_depth, const bns_options *base, int32_t trials,
                        bns_options *best);

/* Measures the device's LDS increment throughput: a reference for reports on
 * the counting step (Section IV-A, step (i)), whose work is one increment of
 * an LDS table word per sample and test; not used by the search.  Four
 * workgroups of 256 lanes per compute unit add 1 to words of an LDS table,
 * the lanes of a wave on different words (as the lane-interleaved replicas
 * of the counting tables), about 17 G increments, timed with events on the
 * library's stream of the device (a few ms; the call returns when they are
 * done).  per_second (required): increments per second over the device;
 * per_cu_per_clock (may be NULL): the same per compute unit and cycle of the
 * device's reported peak clock.  Errors: BNS_E_INVALID_ARG (NULL
 * per_second), BNS_E_DEVICE (a HIP call failed). */
bns_status bns_lds_increment_rate(int32_t device, double *per_second, double *per_cu_per_clock);

int32_t bns_skeleton_n_vars(const bns_skeleton *sk);

/* adj: n_vars * n_vars uint8, adj[i * n + j] = 1 iff edge i - j survived. */
bns_status bns_skeleton_adjacency(const bns_skeleton *sk, uint8_t *adj);

/* Sepset of pair (i, j) (either order).  *len = -1 when the edge was kept,
 * else its size (= removal depth); up to cap members written, ascending.
 * removal_depth may be NULL. */
bns_status bns_skeleton_sepset(const bns_skeleton *sk, int32_t i, int32_t j, int32_t *members,
                               int32_t cap, int32_t *len, int32_t *removal_depth);

/* Bulk export: depth[i * n + j] = removal depth or -1 (n_vars * n_vars int32);
 * sep_off[i * n + j] = offset of the pair's sepset in pool or -1; pool receives
 * up to pool_cap members; *pool_len = members needed.  depth, sep_off and pool
 * may each be NULL. */
bns_status bns_skeleton_removals(const bns_skeleton *sk, int32_t *depth, int64_t *sep_off,
                                 int32_t *pool, int64_t pool_cap, int64_t *pool_len);

/* Per-depth counters; up to cap entries written, *n_depths = depths run.
 * For a handle of bns_pc_skeleton_batch the counters are that problem's own
 * (its edges, tests, removals and re-checks; operand_bytes from its sample
 * count), for its depths up to the last one at which it had a test; the
 * timing fields (kernel_seconds, span_seconds) are those of the batch's
 * launch of that depth, shared by all problems of the batch. */
bns_status bns_skeleton_stats(const bns_skeleton *sk, bns_depth_stats *out, int32_t cap,
                              int32_t *n_depths);

/* A skeleton handle from host arrays (e.g. to orient a skeleton learned
 * elsewhere): adj (n * n uint8, symmetric, 0/1, zero diagonal), depth (n * n
 * int32: removal depth of each removed pair, -1 for kept edges, symmetric),
 * sep_off (n * n int64: for a pair removed at depth d >= 1, the offset of its
 * d sepset members in pool, ascending ids other than the pair; unused
 * otherwise).  The arrays are copied; inconsistent input gives
 * BNS_E_INVALID_ARG.  No device work; the handle has no per-depth counters. */
bns_status bns_skeleton_create(int32_t n_vars, const uint8_t *adj, const int32_t *depth,
                               const int64_t *sep_off, const int32_t *pool, int64_t pool_len,
                               bns_skeleton **out);

/* PC steps 2 and 3 (Section III-C) on a learned skeleton: its CPDAG.
 * Step 2 orients x -> z <- y for every unshielded triple x - z - y (x and y
 * not adjacent) whose middle node z is not in SepSet(x, y); every triple is
 * judged on the skeleton, so the result does not depend on their order, and an
 * edge that two triples orient both ways keeps arrowheads at both ends (a
 * conflict).  Step 3 applies Meek's rules R1-R3 to the undirected edges, with
 * singly-directed edges as premises, in rounds: the orientations a round
 * implies are all found on the graph as it stood and then applied together;
 * an edge one round orients both ways keeps both arrowheads.  cpdag (n_vars *
 * n_vars int8, caller-allocated): cpdag[i * n + j] = 0 when i and j are not
 * adjacent, 1 when they are and the edge has no arrowhead at j, 2 when it has
 * one at j: i -> j is 2 / 1, an undirected edge 1 / 1, a conflict 2 / 2.
 * Runs on the host; the handle is not modified. */
bns_status bns_skeleton_orient(const bns_skeleton *sk, int8_t *cpdag);

void bns_skeleton_free(bns_skeleton *sk);

#ifdef __cplusplus
}
#endif
#endif /* BNS_H */
