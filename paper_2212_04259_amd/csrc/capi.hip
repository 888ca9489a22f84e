// C ABI of the gfx950 G^2 CI-test engine (include/bns.h): argument checks,
// device-resident datasets, the batched per-depth driver of PC-stable
// (Algorithm 1), the plain per-test driver and the CI-batch entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/bns.h"
#include "bns_internal.h"
#include "kernels.h"
#include "skeleton.h"

using namespace bns;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err = "no error";

static bns_status fail(bns_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            return fail(e_ == hipErrorOutOfMemory ? BNS_E_NOMEM : BNS_E_DEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                 \
        }                                                                                  \
    } while (0)

extern "C" const char *bns_last_error(void) { return g_err.c_str(); }

extern "C" void bns_options_default(bns_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->form = BNS_FORM_BATCHED;
    o->precision = BNS_PREC_FP32_RECHECK;
    o->recheck_band = 1e-3;
    o->lds_bytes = 0;
    o->wg_per_cu = 0;
    o->use_graph = 1;
    o->timing = 0;
    o->split_min_samples = 0;
    o->units_per_group = 0;
    o->test_group = 0;
    o->stream = nullptr;
}

static bns_status read_options(const bns_options *in, bns_options *out) {
    bns_options_default(out);
    if (!in) return BNS_OK;
    *out = *in;
    if (out->form != BNS_FORM_BATCHED && out->form != BNS_FORM_PLAIN && out->form != BNS_FORM_EDGE)
        return fail(BNS_E_INVALID_ARG, "options.form must be a BNS_FORM_* value");
    if (out->precision != BNS_PREC_FP32_RECHECK && out->precision != BNS_PREC_FP64)
        return fail(BNS_E_INVALID_ARG, "options.precision must be a BNS_PREC_* value");
    if (!(out->recheck_band >= 0.0) || out->recheck_band > 1.0)
        return fail(BNS_E_INVALID_ARG, "options.recheck_band must be in [0, 1]");
    if (out->lds_bytes < 0 || out->lds_bytes > (160 << 10))
        return fail(BNS_E_INVALID_ARG, "options.lds_bytes must be in [0, 163840]");
    if (out->wg_per_cu < 0 || out->wg_per_cu > 64)
        return fail(BNS_E_INVALID_ARG, "options.wg_per_cu must be in [0, 64]");
    if (out->split_min_samples < -1)
        return fail(BNS_E_INVALID_ARG, "options.split_min_samples must be -1, 0 or positive");
    if (out->units_per_group < 0 || out->units_per_group > 1024)
        return fail(BNS_E_INVALID_ARG, "options.units_per_group must be in [0, 1024]");
    if (out->test_group < 0 || out->test_group > 2)
        return fail(BNS_E_INVALID_ARG, "options.test_group must be 0, 1 or 2");
    if (out->max_replicas < 0 || out->max_replicas > 64 ||
        (out->max_replicas & (out->max_replicas - 1)) != 0)
        return fail(BNS_E_INVALID_ARG, "options.max_replicas must be 0 or a power of two up to 64");
    if (out->tickets_per_grab < 0 || out->tickets_per_grab > kSlotsPerWave)
        return fail(BNS_E_INVALID_ARG, "options.tickets_per_grab must be in [0, %d]", kSlotsPerWave);
    if (out->ticket_runs < 0 || out->ticket_runs > 2)
        return fail(BNS_E_INVALID_ARG, "options.ticket_runs must be 0, 1 or 2");
    if ((out->wave_depths & out->block_depths) != 0u)
        return fail(BNS_E_INVALID_ARG, "options.wave_depths and options.block_depths share a depth");
    if (out->report_errors < 0 || out->report_errors > 1)
        return fail(BNS_E_INVALID_ARG, "options.report_errors must be 0 or 1");
    if (out->workspace_mb < 0) return fail(BNS_E_INVALID_ARG, "options.workspace_mb must be >= 0");
    if (out->statistic != BNS_STAT_G2 && out->statistic != BNS_STAT_X2)
        return fail(BNS_E_INVALID_ARG, "options.statistic must be a BNS_STAT_* value");
    if (out->df_rule != BNS_DF_DECLARED && out->df_rule != BNS_DF_ADJUSTED)
        return fail(BNS_E_INVALID_ARG, "options.df_rule must be a BNS_DF_* value");
    if (out->depth0 < BNS_DEPTH0_AUTO || out->depth0 > BNS_DEPTH0_PAIRS)
        return fail(BNS_E_INVALID_ARG, "options.depth0 must be a BNS_DEPTH0_* value");
    if (out->round_tests < 0 || out->round_tests > 65536)
        return fail(BNS_E_INVALID_ARG, "options.round_tests must be in [0, 65536]");
    if (out->depth1 < BNS_DEPTH1_AUTO || out->depth1 > BNS_DEPTH1_GRAM)
        return fail(BNS_E_INVALID_ARG, "options.depth1 must be a BNS_DEPTH1_* value");
    if (out->group_tests < BNS_GROUP_AUTO || out->group_tests > BNS_GROUP_EDGE)
        return fail(BNS_E_INVALID_ARG, "options.group_tests must be a BNS_GROUP_* value");
    return BNS_OK;
}

// ---------------------------------------------------------------------------
// Device buffers
// ---------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t ensure(size_t n) {
        if (n <= bytes && p) return hipSuccess;
        release();
        size_t want = std::max<size_t>(n, 256);
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) bytes = want;
        return e;
    }
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

struct GraphEntry {
    DepthArgs args;
    int grid = 0;
    int K = 0;
    bool init = false;  // begins with the search's initialisation
    int tri_seq = -1;   // depth sequence that runs depth 1 through the Gram contraction
    uint32_t seq_units = 0;  // work units of each depth sequence's test kernel (2 bits each)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;  // recorded after each replay
    ~GraphEntry() {
        if (done) {
            (void)hipEventSynchronize(done);
            (void)hipEventDestroy(done);
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

// Per-device state: properties, a library stream, and grow-only workspaces.
struct DevCtx {
    int device = -1;
    int num_cu = 0;
    int max_lds_block = 0;
    hipStream_t stream = nullptr;
    std::mutex mu;
    // skeleton search
    DevBuf setup, adj, adjbits, nbr, ipos, deg, rowcnt, rowbase, edges_tmp, edges, min_accept, rdepth, pool, ctl;
    DevBuf pstat, ecnt;  // per-problem counters of multi-dataset searches
    DevBuf pair_part;    // partial Gram tiles of depth 0 through the pair contraction
    DevBuf tri_node, tri_rowoff, tri_eidx, tri_part;  // depth 1 through the masked contractions
    DevBuf pairs_setup, pairs_out;  // bns_ci_pairs: tile plan and results
    DevBuf err_val, err_tag, err_cnt;  // verification log
    std::vector<uint64_t> binom_host;  // C(n, k) rows built so far (host)
    // bytes of the last search set-up uploaded into `setup` (a repeated
    // search skips the upload)
    std::vector<char> setup_last;
    void *setup_last_dev = nullptr;
    // merge tables and chunk counters of split depths: all zero between tests
    DevBuf split_tab, split_cnt;
    bool split_dirty = false;
    // CI batch and plain form
    DevBuf ci_tests, ci_z, ci_out, ci_tab, ci_taboff, plain_part, plain_ws, plain_out;
    CiOutDev *h_out = nullptr;  // pinned readback slot
    Ctl *h_ctl = nullptr;       // pinned control-block readback
    // launch completion: the publishing kernel counts launches in pub (device:
    // sequence, workgroup counter) and writes the count into h_flag (pinned)
    unsigned long long *h_flag = nullptr;
    void *pub = nullptr;
    unsigned long long pub_expected = 0;
    void *hpin = nullptr;       // pinned staging for uploads and result downloads
    size_t hpin_bytes = 0;
    hipError_t pinned(size_t n) {
        if (n <= hpin_bytes && hpin) return hipSuccess;
        if (hpin) (void)hipHostFree(hpin);
        hpin = nullptr;
        hpin_bytes = 0;
        const size_t want = std::max<size_t>(n, 1 << 16);
        hipError_t e = hipHostMalloc(&hpin, want, hipHostMallocDefault);
        if (e == hipSuccess) hpin_bytes = want;
        return e;
    }
    std::vector<std::unique_ptr<GraphEntry>> graphs;  // captured depth launches
    int search_lds = 0;  // default dynamic LDS of the skeleton test kernel (bytes)
    int last_sequences = 0;  // depth sequences the last finished search needed
    void *hres = nullptr;    // pinned staging for result downloads
    size_t hres_bytes = 0;
    hipError_t results(size_t n) {
        if (n <= hres_bytes && hres) return hipSuccess;
        if (hres) (void)hipHostFree(hres);
        hres = nullptr;
        hres_bytes = 0;
        const size_t want = std::max<size_t>(n, 1 << 16);
        hipError_t e = hipHostMalloc(&hres, want, hipHostMallocDefault);
        if (e == hipSuccess) hres_bytes = want;
        return e;
    }
    int lds_per_cu = 0;
    int wall_khz = 0;  // device wall-clock rate
};

static std::mutex g_ctx_mu;
static std::vector<std::unique_ptr<DevCtx>> g_ctx;

static bns_status get_ctx(int device, DevCtx **out) {
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    for (auto &c : g_ctx)
        if (c->device == device) {
            *out = c.get();
            return BNS_OK;
        }
    auto c = std::make_unique<DevCtx>();
    c->device = device;
    HIP_TRY(hipSetDevice(device));
    HIP_TRY(hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, device));
    HIP_TRY(hipDeviceGetAttribute(&c->max_lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                  device));
    HIP_TRY(hipDeviceGetAttribute(&c->lds_per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                  device));
    if (hipDeviceGetAttribute(&c->wall_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess ||
        c->wall_khz <= 0)
        c->wall_khz = 100000;
    HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    HIP_TRY(hipHostMalloc((void **)&c->h_out, sizeof(CiOutDev), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void **)&c->h_ctl, sizeof(Ctl), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void **)&c->h_flag, 64, hipHostMallocDefault));
    *c->h_flag = 0;
    HIP_TRY(hipMalloc(&c->pub, 64));
    HIP_TRY(hipMemset(c->pub, 0, 64));
    *out = c.get();
    g_ctx.push_back(std::move(c));
    return BNS_OK;
}

// Switches to a device for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess) ok = true;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// ---------------------------------------------------------------------------
// Datasets
// ---------------------------------------------------------------------------
struct bns_dataset {
    int device = -1;
    const uint8_t *d_data = nullptr;
    bool owns = false;
    int64_t ld = 0;
    int64_t m = 0;
    int32_t n = 0;
    std::vector<uint8_t> cards;
    uint8_t *d_cards = nullptr;
    ~bns_dataset() {
        if (owns && d_data) (void)hipFree((void *)d_data);
        if (d_cards) (void)hipFree(d_cards);
    }
};

static bns_status check_shape(int64_t m, int32_t n, const uint8_t *cards) {
    if (m < 1 || m > INT32_MAX) return fail(BNS_E_INVALID_ARG, "n_samples must be in [1, 2^31-1]");
    if (n < 2 || n > 65535) return fail(BNS_E_INVALID_ARG, "n_vars must be in [2, 65535]");
    if (!cards) return fail(BNS_E_INVALID_ARG, "cards is NULL");
    for (int32_t v = 0; v < n; ++v)
        if (cards[v] == 0) return fail(BNS_E_INVALID_ARG, "cards[%d] is 0", v);
    return BNS_OK;
}

static bns_status upload_cards(bns_dataset *ds, const uint8_t *cards) {
    ds->cards.assign(cards, cards + ds->n);
    HIP_TRY(hipMalloc((void **)&ds->d_cards, (size_t)ds->n));
    HIP_TRY(hipMemcpy(ds->d_cards, cards, (size_t)ds->n, hipMemcpyHostToDevice));
    return BNS_OK;
}

extern "C" bns_status bns_dataset_create(const uint8_t *data, int64_t m, int32_t n,
                                         const uint8_t *cards, bns_dataset **out) {
    if (!out) return fail(BNS_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!data) return fail(BNS_E_INVALID_ARG, "data is NULL");
    bns_status st = check_shape(m, n, cards);
    if (st != BNS_OK) return st;
    for (int32_t v = 0; v < n; ++v) {
        const uint8_t *col = data + (int64_t)v * m;
        const uint8_t r = cards[v];
        for (int64_t s = 0; s < m; ++s)
            if (col[s] >= r)
                return fail(BNS_E_VALUE_RANGE, "value %u of variable %d at sample %lld >= card %u",
                            (unsigned)col[s], v, (long long)s, (unsigned)r);
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::unique_ptr<bns_dataset> ds(new bns_dataset());
    ds->device = dev;
    ds->m = m;
    ds->n = n;
    ds->ld = (m + 255) / 256 * 256;
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, (size_t)ds->ld * (size_t)n));
    ds->d_data = (const uint8_t *)p;
    ds->owns = true;
    HIP_TRY(hipMemset(p, 0, (size_t)ds->ld * (size_t)n));
    HIP_TRY(hipMemcpy2D(p, (size_t)ds->ld, data, (size_t)m, (size_t)m, (size_t)n,
                        hipMemcpyHostToDevice));
    st = upload_cards(ds.get(), cards);
    if (st != BNS_OK) return st;
    *out = ds.release();
    return BNS_OK;
}

extern "C" bns_status bns_dataset_wrap_device(const uint8_t *d_data, int64_t ld, int64_t m,
                                              int32_t n, const uint8_t *cards, bns_dataset **out) {
    if (!out) return fail(BNS_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!d_data) return fail(BNS_E_INVALID_ARG, "d_data is NULL");
    bns_status st = check_shape(m, n, cards);
    if (st != BNS_OK) return st;
    if (ld < m || (ld % 16) != 0) return fail(BNS_E_INVALID_ARG, "ld must be >= n_samples and a multiple of 16");
    if (((uintptr_t)d_data % 16) != 0) return fail(BNS_E_INVALID_ARG, "d_data must be 16-byte aligned");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::unique_ptr<bns_dataset> ds(new bns_dataset());
    ds->device = dev;
    ds->m = m;
    ds->n = n;
    ds->ld = ld;
    ds->d_data = d_data;
    ds->owns = false;
    st = upload_cards(ds.get(), cards);
    if (st != BNS_OK) return st;
    DevCtx *dc = nullptr;
    st = get_ctx(dev, &dc);
    if (st != BNS_OK) return st;
    std::lock_guard<std::mutex> lk(dc->mu);
    unsigned long long *bad = nullptr;
    HIP_TRY(hipMalloc((void **)&bad, sizeof(unsigned long long)));
    const unsigned long long init = ~0ull;
    unsigned long long hbad = ~0ull;
    hipError_t e = hipMemcpy(bad, &init, sizeof(init), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_validate(d_data, ld, m, n, ds->d_cards, bad, dc->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, dc->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(dc->stream);
    (void)hipFree(bad);
    HIP_TRY(e);
    if (hbad != ~0ull) {
        const int64_t v = (int64_t)(hbad / (unsigned long long)m), s = (int64_t)(hbad % (unsigned long long)m);
        return fail(BNS_E_VALUE_RANGE, "value of variable %lld at sample %lld >= card %u", (long long)v,
                    (long long)s, (unsigned)cards[v]);
    }
    *out = ds.release();
    return BNS_OK;
}

extern "C" void bns_dataset_free(bns_dataset *ds) { delete ds; }

// Device workspace a call needs against options.workspace_mb.
static bns_status check_workspace(const bns_options &o, double need_bytes, const char *what) {
    if (o.workspace_mb > 0 && need_bytes > (double)o.workspace_mb * 1048576.0)
        return fail(BNS_E_NOMEM, "%s needs %.1f MiB of device workspace, above options.workspace_mb = %d",
                    what, need_bytes / 1048576.0, o.workspace_mb);
    return BNS_OK;
}

// ---------------------------------------------------------------------------
// Tiles
// ---------------------------------------------------------------------------
static const int kDefaultLdsBytes = 40 << 10;

// Tile of a launch from the options and the device's LDS per workgroup;
// default_lds: the dynamic LDS used when the options leave it open.
static bns_status make_tile_for(int max_lds_block, int default_lds, const bns_options &o, Tile *t) {
    int lds = o.lds_bytes ? o.lds_bytes : default_lds;
    const int static_reserve = 4096;  // TestSh + TicketSh + reductions
    if (lds + static_reserve > max_lds_block) lds = max_lds_block - static_reserve;
    lds &= ~255;
    if (lds < 4096) return fail(BNS_E_DEVICE, "device LDS per workgroup too small (%d bytes)", max_lds_block);
    if (lds > (64 << 10) - static_reserve) {
        hipError_t e = allow_dynamic_lds(lds);
        if (e != hipSuccess) return fail(BNS_E_DEVICE, "cannot enable %d bytes of dynamic LDS: %s", lds, hipGetErrorString(e));
    }
    t->lds_words = lds / 4;
    t->max_rep_log2 = 5;  // 32 copies: fewer to clear and sum than 64, as fast to count
    if (o.max_replicas > 0) t->max_rep_log2 = __builtin_ctz((unsigned)o.max_replicas);
    t->fp64 = (o.precision == BNS_PREC_FP64) ? 1 : 0;
    t->band = o.recheck_band;
    t->stat = (int16_t)o.statistic;
    t->df_rule = (int16_t)o.df_rule;
    return BNS_OK;
}

static bns_status make_tile(const DevCtx &dc, const bns_options &o, Tile *t, bool search = false) {
    return make_tile_for(dc.max_lds_block, search && dc.search_lds ? dc.search_lds : kDefaultLdsBytes, o, t);
}

static bns_status check_table(const std::vector<uint8_t> &cards, int x, int y, const int32_t *z,
                              int nz, const Tile &tile) {
    uint64_t rxy = (uint64_t)cards[x] * cards[y];
    uint64_t T = rxy;
    for (int k = 0; k < nz; ++k) {
        T *= cards[z[k]];
        if (T > kMaxCells) return fail(BNS_E_TABLE_TOO_LARGE, "table of test %d-%d exceeds %u cells", x, y, kMaxCells);
    }
    // one stratum (table + marginals) plus the spill words must fit a wave's slice
    if (rxy + cards[x] + cards[y] + 1 + 64 > (uint64_t)(tile.lds_words / kWaves))
        return fail(BNS_E_TABLE_TOO_LARGE, "r_x * r_y of test %d-%d exceeds the LDS budget", x, y);
    return BNS_OK;
}

// Host-side checks of a batch of CI tests (ids, disjointness, table sizes).
static bns_status check_ci_tests(const bns_dataset *ds, const bns_ci_test *tests, int64_t n_tests,
                                 const int32_t *z_pool, int64_t z_pool_len, const Tile &tile) {
    const int n = ds->n;
    for (int64_t t = 0; t < n_tests; ++t) {
        const bns_ci_test &q = tests[t];
        if (q.x < 0 || q.x >= n || q.y < 0 || q.y >= n || q.x == q.y)
            return fail(BNS_E_INVALID_ARG, "test %lld: bad x/y", (long long)t);
        if (q.n_z < 0 || q.n_z > kMaxZ) return fail(BNS_E_INVALID_ARG, "test %lld: n_z out of [0, %d]", (long long)t, kMaxZ);
        if (q.n_z > 0 && (q.z_offset < 0 || (int64_t)q.z_offset + q.n_z > z_pool_len))
            return fail(BNS_E_INVALID_ARG, "test %lld: z range outside z_pool", (long long)t);
        for (int k = 0; k < q.n_z; ++k) {
            const int32_t zv = z_pool[q.z_offset + k];
            if (zv < 0 || zv >= n || zv == q.x || zv == q.y)
                return fail(BNS_E_INVALID_ARG, "test %lld: bad conditioning variable %d", (long long)t, zv);
        }
        bns_status st = check_table(ds->cards, q.x, q.y, q.n_z ? z_pool + q.z_offset : nullptr, q.n_z, tile);
        if (st != BNS_OK) return st;
    }
    return BNS_OK;
}

// ---------------------------------------------------------------------------
// bns_ci_batch
// ---------------------------------------------------------------------------
extern "C" bns_status bns_ci_batch(const bns_dataset *ds, const bns_ci_test *tests, int64_t n_tests,
                                   const int32_t *z_pool, int64_t z_pool_len, double alpha,
                                   const bns_options *opt, double *g2, int64_t *df, double *p,
                                   int32_t *flags, int32_t *tables_out,
                                   const int64_t *table_offsets) {
    if (!ds) return fail(BNS_E_INVALID_ARG, "dataset is NULL");
    if (n_tests < 0) return fail(BNS_E_INVALID_ARG, "n_tests < 0");
    if (n_tests > 0 && !tests) return fail(BNS_E_INVALID_ARG, "tests is NULL");
    if (z_pool_len < 0 || (z_pool_len > 0 && !z_pool)) return fail(BNS_E_INVALID_ARG, "bad z_pool");
    if (!(alpha > 0.0 && alpha < 1.0)) return fail(BNS_E_INVALID_ARG, "alpha must be in (0, 1)");
    if (tables_out && !table_offsets) return fail(BNS_E_INVALID_ARG, "tables_out needs table_offsets");
    bns_options o;
    bns_status st = read_options(opt, &o);
    if (st != BNS_OK) return st;
    if (n_tests == 0) return BNS_OK;
    DevCtx *dc = nullptr;
    st = get_ctx(ds->device, &dc);
    if (st != BNS_OK) return st;
    Tile tile;
    st = make_tile(*dc, o, &tile);
    if (st != BNS_OK) return st;
    st = check_ci_tests(ds, tests, n_tests, z_pool, z_pool_len, tile);
    if (st != BNS_OK) return st;
    {
        double need = (double)(sizeof(CiTestDev) + sizeof(CiOutDev)) * (double)n_tests +
                      4.0 * (double)std::max<int64_t>(z_pool_len, 1);
        if (tables_out) {
            int64_t tab_words = 0;
            for (int64_t t = 0; t < n_tests; ++t) {
                int64_t T = (int64_t)ds->cards[tests[t].x] * ds->cards[tests[t].y];
                for (int k = 0; k < tests[t].n_z; ++k) T *= ds->cards[z_pool[tests[t].z_offset + k]];
                tab_words = std::max(tab_words, table_offsets[t] + T);
            }
            need += 4.0 * (double)tab_words + 8.0 * (double)n_tests;
        }
        st = check_workspace(o, need, "bns_ci_batch");
        if (st != BNS_OK) return st;
    }
    DeviceGuard dg(ds->device);
    if (!dg.ok) return fail(BNS_E_DEVICE, "cannot select device %d", ds->device);
    std::lock_guard<std::mutex> lk(dc->mu);
    hipStream_t s = o.stream ? (hipStream_t)o.stream : dc->stream;
    HIP_TRY(dc->ci_tests.ensure(sizeof(CiTestDev) * (size_t)n_tests));
    HIP_TRY(dc->ci_z.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(z_pool_len, 1)));
    HIP_TRY(dc->ci_out.ensure(sizeof(CiOutDev) * (size_t)n_tests));
    std::vector<CiTestDev> ht((size_t)n_tests);
    int64_t tab_total = 0;
    for (int64_t t = 0; t < n_tests; ++t) {
        ht[t] = {tests[t].x, tests[t].y, tests[t].n_z, tests[t].z_offset};
        if (tables_out) {
            int64_t T = (int64_t)ds->cards[tests[t].x] * ds->cards[tests[t].y];
            for (int k = 0; k < tests[t].n_z; ++k) T *= ds->cards[z_pool[tests[t].z_offset + k]];
            if (table_offsets[t] < 0) return fail(BNS_E_INVALID_ARG, "negative table offset");
            tab_total = std::max(tab_total, table_offsets[t] + T);
        }
    }
    HIP_TRY(hipMemcpyAsync(dc->ci_tests.p, ht.data(), sizeof(CiTestDev) * (size_t)n_tests,
                           hipMemcpyHostToDevice, s));
    if (z_pool_len > 0)
        HIP_TRY(hipMemcpyAsync(dc->ci_z.p, z_pool, sizeof(int32_t) * (size_t)z_pool_len,
                               hipMemcpyHostToDevice, s));
    uint32_t *d_tab = nullptr;
    const int64_t *d_taboff = nullptr;
    if (tables_out) {
        HIP_TRY(dc->ci_tab.ensure(sizeof(uint32_t) * (size_t)tab_total));
        HIP_TRY(dc->ci_taboff.ensure(sizeof(int64_t) * (size_t)n_tests));
        HIP_TRY(hipMemcpyAsync(dc->ci_taboff.p, table_offsets, sizeof(int64_t) * (size_t)n_tests,
                               hipMemcpyHostToDevice, s));
        d_tab = dc->ci_tab.as<uint32_t>();
        d_taboff = dc->ci_taboff.as<int64_t>();
    }
    const int wg = std::max(1, depth_tests_max_wg_per_cu(tile.lds_words * 4));
    const int grid = (int)std::min<int64_t>((n_tests + kWaves - 1) / kWaves, (int64_t)dc->num_cu * wg);
    HIP_TRY(launch_ci_batch(ds->d_data, ds->ld, ds->m, ds->d_cards, dc->ci_tests.as<CiTestDev>(),
                            dc->ci_z.as<int32_t>(), n_tests, alpha, tile, dc->ci_out.as<CiOutDev>(),
                            d_tab, d_taboff, grid, s));
    std::vector<CiOutDev> ho((size_t)n_tests);
    HIP_TRY(hipMemcpyAsync(ho.data(), dc->ci_out.p, sizeof(CiOutDev) * (size_t)n_tests,
                           hipMemcpyDeviceToHost, s));
    if (tables_out)
        HIP_TRY(hipMemcpyAsync(tables_out, d_tab, sizeof(uint32_t) * (size_t)tab_total,
                               hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int64_t t = 0; t < n_tests; ++t) {
        if (ho[t].flags >> 8) return fail(BNS_E_TABLE_TOO_LARGE, "test %lld exceeded device limits", (long long)t);
        if (g2) g2[t] = ho[t].g2;
        if (df) df[t] = ho[t].df;
        if (p) p[t] = ho[t].p;
        if (flags) flags[t] = ho[t].flags & 3;
    }
    return BNS_OK;
}

// ---------------------------------------------------------------------------
// bns_ci_batch_noalloc: the same tests with no allocation.  The tests, the
// conditioning pool and the results are staged in `scratch`, a fixed device
// array of the library (one copy per device, held until the process ends).
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address comes from hipGetSymbolAddress, once per device with that
// device current, and only that address is used.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[BNS_NOALLOC_SCRATCH_BYTES];

static const int kNoallocDevices = 64;
static std::mutex g_noalloc_mu[kNoallocDevices];   // serialises calls per device
static void *g_scratch_dev[kNoallocDevices];       // device address of scratch, per device
static int g_noalloc_cu[kNoallocDevices], g_noalloc_lds[kNoallocDevices];

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

extern "C" bns_status bns_ci_batch_noalloc(const bns_dataset *ds, const bns_ci_test *tests, int64_t n_tests,
                                           const int32_t *z_pool, int64_t z_pool_len, double alpha,
                                           const bns_options *opt, double *g2, int64_t *df, double *p,
                                           int32_t *flags) {
    static_assert(sizeof(bns_ci_test) == sizeof(CiTestDev), "test records are copied as they are");
    if (!ds) return fail(BNS_E_INVALID_ARG, "dataset is NULL");
    if (n_tests < 0) return fail(BNS_E_INVALID_ARG, "n_tests < 0");
    if (n_tests > 0 && !tests) return fail(BNS_E_INVALID_ARG, "tests is NULL");
    if (z_pool_len < 0 || (z_pool_len > 0 && !z_pool)) return fail(BNS_E_INVALID_ARG, "bad z_pool");
    if (!(alpha > 0.0 && alpha < 1.0)) return fail(BNS_E_INVALID_ARG, "alpha must be in (0, 1)");
    if (ds->device < 0 || ds->device >= kNoallocDevices) return fail(BNS_E_DEVICE, "device %d out of range", ds->device);
    bns_options o;
    bns_status st = read_options(opt, &o);
    if (st != BNS_OK) return st;
    if (n_tests == 0) return BNS_OK;
    // scratch layout: tests | conditioning pool | g2 | p | df | flags
    const size_t o_z = al256(sizeof(CiTestDev) * (size_t)n_tests);
    const size_t o_g2 = o_z + al256(sizeof(int32_t) * (size_t)z_pool_len);
    const size_t o_p = o_g2 + al256(sizeof(double) * (size_t)n_tests);
    const size_t o_df = o_p + al256(sizeof(double) * (size_t)n_tests);
    const size_t o_fl = o_df + al256(sizeof(int64_t) * (size_t)n_tests);
    const size_t need = o_fl + al256(sizeof(int32_t) * (size_t)n_tests);
    if (need > (size_t)BNS_NOALLOC_SCRATCH_BYTES)
        return fail(BNS_E_NOMEM, "bns_ci_batch_noalloc: %lld tests with %lld pool entries need %zu bytes of "
                    "scratch, above the fixed %d", (long long)n_tests, (long long)z_pool_len, need,
                    BNS_NOALLOC_SCRATCH_BYTES);
    const int dev = ds->device;
    std::lock_guard<std::mutex> lk(g_noalloc_mu[dev]);
    DeviceGuard dg(dev);
    if (!dg.ok) return fail(BNS_E_DEVICE, "cannot select device %d", dev);
    if (!g_scratch_dev[dev]) {
        // first call on this device (now current): the device copy's address
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        HIP_TRY(hipDeviceGetAttribute(&g_noalloc_cu[dev], hipDeviceAttributeMultiprocessorCount, dev));
        HIP_TRY(hipDeviceGetAttribute(&g_noalloc_lds[dev], hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        g_scratch_dev[dev] = ptr;
    }
    Tile tile;
    st = make_tile_for(g_noalloc_lds[dev], kDefaultLdsBytes, o, &tile);
    if (st != BNS_OK) return st;
    st = check_ci_tests(ds, tests, n_tests, z_pool, z_pool_len, tile);
    if (st != BNS_OK) return st;
    char *base = (char *)g_scratch_dev[dev];
    hipStream_t s = (hipStream_t)o.stream;
    HIP_TRY(hipMemcpyAsync(base, tests, sizeof(CiTestDev) * (size_t)n_tests, hipMemcpyHostToDevice, s));
    if (z_pool_len > 0)
        HIP_TRY(hipMemcpyAsync(base + o_z, z_pool, sizeof(int32_t) * (size_t)z_pool_len, hipMemcpyHostToDevice, s));
    CiOutSoa soa{(double *)(base + o_g2), (double *)(base + o_p), (int64_t *)(base + o_df),
                 (int32_t *)(base + o_fl)};
    const int wg = std::max(1, depth_tests_max_wg_per_cu(tile.lds_words * 4));
    const int grid = (int)std::min<int64_t>((n_tests + kWaves - 1) / kWaves, (int64_t)g_noalloc_cu[dev] * wg);
    HIP_TRY(launch_ci_batch(ds->d_data, ds->ld, ds->m, ds->d_cards, (const CiTestDev *)base,
                            (const int32_t *)(base + o_z), n_tests, alpha, tile, nullptr, nullptr, nullptr,
                            grid, s, soa));
    if (g2) HIP_TRY(hipMemcpyAsync(g2, soa.g2, sizeof(double) * (size_t)n_tests, hipMemcpyDeviceToHost, s));
    if (p) HIP_TRY(hipMemcpyAsync(p, soa.p, sizeof(double) * (size_t)n_tests, hipMemcpyDeviceToHost, s));
    if (df) HIP_TRY(hipMemcpyAsync(df, soa.df, sizeof(int64_t) * (size_t)n_tests, hipMemcpyDeviceToHost, s));
    if (flags) HIP_TRY(hipMemcpyAsync(flags, soa.flags, sizeof(int32_t) * (size_t)n_tests, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (flags)
        for (int64_t t = 0; t < n_tests; ++t) {
            if (flags[t] >> 8) return fail(BNS_E_TABLE_TOO_LARGE, "test %lld exceeded device limits", (long long)t);
            flags[t] &= 3;
        }
    return BNS_OK;
}

// Depth 0 through the pair contraction: one-hot column maps, tiles and
// sample chunks of every problem.
struct PairPlan {
    bool on = false;
    int T = 64;
    int64_t chunk = 0, items = 0, tiles = 0, part_bytes = 0, gram_bytes = 0;
    std::vector<GramProb> gps;
    std::vector<int32_t> oh_var, var_oh;
    std::vector<uint16_t> oh_cat;
};
// Partial tiles held at most by the pair contraction (beyond it, depth 0
// runs in the test kernel, or a forced pair path fails with BNS_E_NOMEM).
static const int64_t kPairPartMax = 1ll << 30;
// Depth 0 through the contraction in automatic mode from this many
// pair-samples (pairs times samples summed over the problems) on: measured on
// MI355X, 8.9e7 (60 variables, 50,000 samples) is faster in the test kernel,
// 2.4e9 (220 variables, 100,000 samples) and more through the contraction.
static const double kPairsAutoWork = 5e8;
// Depth 1 through the masked contractions: work items held at most (64 KiB
// each; beyond, the depth runs in the test kernel).
static const int64_t kTriItemsMax = 16384;

static bns_status plan_pairs(const DevCtx &dc, const bns_dataset *const *ds, int32_t P, PairPlan &pp) {
    pp = PairPlan();
    int64_t m_max = 1;
    for (int32_t k = 0; k < P; ++k) m_max = std::max(m_max, ds[k]->m);
    // 64 x 64 tiles: a workgroup's LDS (two steps of 2 x 64 one-hot columns)
    // leaves room for more workgroups per CU than 128 x 128 tiles do, which
    // the expansion and LDS traffic need more than the larger tiles' reuse
    // (1,000 variables: 3.91 -> 3.46 ms; 64 datasets: 3.01 -> 2.58 ms)
    pp.T = 64;
    const int64_t T = pp.T;
    int64_t tiles = 0;
    std::vector<int64_t> tiles_k((size_t)P);
    for (int32_t k = 0; k < P; ++k) {
        int64_t R = 0;
        for (uint8_t c : ds[k]->cards) R += c;
        const int64_t nb = (R + T - 1) / T;
        tiles_k[k] = nb * (nb + 1) / 2;
        tiles += tiles_k[k];
    }
    // about two work items per workgroup slot of the device: split the
    // samples into chunks when the tiles alone are fewer
    const int64_t want = 2ll * dc.num_cu * gram_max_wg_per_cu(pp.T);
    int64_t chunk = (m_max + 63) / 64 * 64;
    if (tiles < want) chunk = std::max<int64_t>(2048, ((m_max * tiles + want - 1) / want + 63) / 64 * 64);
    pp.chunk = std::min(chunk, (m_max + 63) / 64 * 64);
    pp.gps.resize((size_t)P);
    pp.var_oh.clear();
    for (int32_t k = 0; k < P; ++k) {
        const bns_dataset *d = ds[k];
        GramProb &g = pp.gps[k];
        g.data = d->d_data;
        g.ld = d->ld;
        g.m = d->m;
        g.oh_base = (int32_t)pp.oh_var.size();
        int32_t R = 0;
        for (int32_t v = 0; v < d->n; ++v) {
            pp.var_oh.push_back(R);
            const uint16_t wide = d->cards[v] > 8 ? 0x100 : 0;
            for (int x = 0; x < d->cards[v]; ++x) {
                pp.oh_var.push_back(v);
                pp.oh_cat.push_back((uint16_t)(x | wide));
            }
            R += d->cards[v];
        }
        const int64_t Rp = (R + T - 1) / T * T;
        for (int64_t c = R; c < Rp; ++c) {
            pp.oh_var.push_back(-1);
            pp.oh_cat.push_back(0);
        }
        g.R = (int32_t)Rp;
        g.nb = (int32_t)(Rp / T);
        g.nchunks = (int32_t)((d->m + pp.chunk - 1) / pp.chunk);
        g.item_base = pp.items;
        g.tile_base = pp.tiles;
        pp.items += tiles_k[k] * g.nchunks;
        pp.tiles += tiles_k[k];
    }
    pp.part_bytes = pp.items * T * T * 4;
    pp.gram_bytes = pp.items > pp.tiles ? pp.tiles * T * T * 4 : 0;  // summed tiles (when chunks were split)
    if (pp.part_bytes + pp.gram_bytes > kPairPartMax || (int64_t)pp.oh_var.size() > INT32_MAX) {
        const double mib = (double)(pp.part_bytes + pp.gram_bytes) / 1048576.0;
        pp = PairPlan();
        return fail(BNS_E_NOMEM, "depth 0 through the pair contraction needs %.0f MiB of partial tiles (limit %lld MiB)",
                    mib, (long long)(kPairPartMax >> 20));
    }
    pp.on = true;
    return BNS_OK;
}

// ---------------------------------------------------------------------------
// bns_ci_pairs: every pairwise marginal test of a dataset through the pair
// contraction.
// ---------------------------------------------------------------------------
extern "C" bns_status bns_ci_pairs(const bns_dataset *ds, double alpha, const bns_options *opt, double *stat,
                                   int64_t *df, double *p, int32_t *flags) {
    if (!ds) return fail(BNS_E_INVALID_ARG, "dataset is NULL");
    if (!(alpha > 0.0 && alpha < 1.0)) return fail(BNS_E_INVALID_ARG, "alpha must be in (0, 1)");
    bns_options o;
    bns_status st = read_options(opt, &o);
    if (st != BNS_OK) return st;
    DevCtx *dc = nullptr;
    st = get_ctx(ds->device, &dc);
    if (st != BNS_OK) return st;
    DeviceGuard dg(ds->device);
    if (!dg.ok) return fail(BNS_E_DEVICE, "cannot select device %d", ds->device);
    std::lock_guard<std::mutex> lk(dc->mu);
    hipStream_t s = o.stream ? (hipStream_t)o.stream : dc->stream;
    PairPlan pp;
    st = plan_pairs(*dc, &ds, 1, pp);
    if (st != BNS_OK) return st;
    const int64_t n = ds->n, npairs = n * (n - 1) / 2;
    auto al8 = [](size_t x) { return (x + 7) & ~(size_t)7; };
    const size_t o_ohvar = al8(sizeof(GramProb));
    const size_t o_ohcat = al8(o_ohvar + sizeof(int32_t) * pp.oh_var.size());
    const size_t o_varoh = al8(o_ohcat + sizeof(uint16_t) * pp.oh_cat.size());
    const size_t setup_bytes = al8(o_varoh + sizeof(int32_t) * pp.var_oh.size());
    const size_t out_bytes = (size_t)npairs * (8 + 8 + 8 + 4) + 32;
    st = check_workspace(o, (double)(setup_bytes + out_bytes + pp.part_bytes + pp.gram_bytes), "bns_ci_pairs");
    if (st != BNS_OK) return st;
    std::vector<char> h(setup_bytes, 0);
    std::memcpy(h.data(), pp.gps.data(), sizeof(GramProb));
    std::memcpy(h.data() + o_ohvar, pp.oh_var.data(), sizeof(int32_t) * pp.oh_var.size());
    std::memcpy(h.data() + o_ohcat, pp.oh_cat.data(), sizeof(uint16_t) * pp.oh_cat.size());
    std::memcpy(h.data() + o_varoh, pp.var_oh.data(), sizeof(int32_t) * pp.var_oh.size());
    HIP_TRY(dc->pairs_setup.ensure(setup_bytes));
    HIP_TRY(dc->pair_part.ensure((size_t)(pp.part_bytes + pp.gram_bytes)));
    HIP_TRY(dc->pairs_out.ensure(out_bytes));
    HIP_TRY(hipMemcpyAsync(dc->pairs_setup.p, h.data(), setup_bytes, hipMemcpyHostToDevice, s));
    char *sb = dc->pairs_setup.as<char>();
    PairArgs pa;
    std::memset(&pa, 0, sizeof(pa));
    pa.gp = (const GramProb *)sb;
    pa.oh_var = (const int32_t *)(sb + o_ohvar);
    pa.oh_cat = (const uint16_t *)(sb + o_ohcat);
    pa.var_oh = (const int32_t *)(sb + o_varoh);
    pa.part = dc->pair_part.as<int32_t>();
    pa.gram = pp.gram_bytes ? pa.part + pp.part_bytes / 4 : pa.part;
    pa.items = pp.items;
    pa.tiles = pp.tiles;
    pa.chunk = pp.chunk;
    pa.T = pp.T;
    pa.n_gp = 1;
    pa.gram_grid = (int)std::min<int64_t>(pp.items, (int64_t)dc->num_cu * gram_max_wg_per_cu(pp.T));
    char *ob = dc->pairs_out.as<char>();
    double *d_stat = (double *)ob;
    double *d_p = d_stat + npairs;
    int64_t *d_df = (int64_t *)(d_p + npairs);
    int32_t *d_fl = (int32_t *)(d_df + npairs);
    HIP_TRY(launch_ci_pairs(pa, ds->d_cards, ds->n, alpha, o.statistic, o.df_rule, d_stat, d_df, d_p, d_fl, s));
    if (stat) HIP_TRY(hipMemcpyAsync(stat, d_stat, sizeof(double) * (size_t)npairs, hipMemcpyDeviceToHost, s));
    if (p) HIP_TRY(hipMemcpyAsync(p, d_p, sizeof(double) * (size_t)npairs, hipMemcpyDeviceToHost, s));
    if (df) HIP_TRY(hipMemcpyAsync(df, d_df, sizeof(int64_t) * (size_t)npairs, hipMemcpyDeviceToHost, s));
    if (flags) HIP_TRY(hipMemcpyAsync(flags, d_fl, sizeof(int32_t) * (size_t)npairs, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return BNS_OK;
}

// ---------------------------------------------------------------------------
// Skeleton results
// ---------------------------------------------------------------------------

extern "C" bns_status bns_lds_increment_rate(int32_t device, double *per_second, double *per_cu_per_clock) {
    if (!per_second) return fail(BNS_E_INVALID_ARG, "per_second is NULL");
    DevCtx *dc = nullptr;
    bns_status st = get_ctx(device, &dc);
    if (st != BNS_OK) return st;
    DeviceGuard dg(device);
    if (!dg.ok) return fail(BNS_E_DEVICE, "cannot select device %d", device);
    std::lock_guard<std::mutex> lk(dc->mu);
    hipStream_t s = dc->stream;
    int clk_khz = 0;
    HIP_TRY(hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeClockRate, device));
    DevBuf sink;
    HIP_TRY(sink.ensure(sizeof(unsigned int)));
    const int grid = 4 * dc->num_cu, steps = 4096;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    struct EvFree {
        hipEvent_t &a, &b;
        ~EvFree() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } evf{e0, e1};
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(launch_lds_rate(grid, steps / 8, sink.as<unsigned int>(), s));  // warm-up
    HIP_TRY(hipEventRecord(e0, s));
    HIP_TRY(launch_lds_rate(grid, steps, sink.as<unsigned int>(), s));
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    if (!(ms > 0.0f)) return fail(BNS_E_DEVICE, "the measurement took no time");
    const double incs = (double)grid * kWG * (double)steps * 16.0;
    *per_second = incs / (ms * 1e-3);
    if (per_cu_per_clock)
        *per_cu_per_clock = clk_khz > 0 ? *per_second / dc->num_cu / (clk_khz * 1e3) : 0.0;
    return BNS_OK;
}

extern "C" int32_t bns_skeleton_n_vars(const bns_skeleton *sk) { return sk ? sk->n : 0; }

extern "C" bns_status bns_skeleton_adjacency(const bns_skeleton *sk, uint8_t *adj) {
    if (!sk || !adj) return fail(BNS_E_INVALID_ARG, "NULL argument");
    sk->expand();
    std::memcpy(adj, sk->adj.data(), sk->adj.size());
    return BNS_OK;
}

extern "C" bns_status bns_skeleton_sepset(const bns_skeleton *sk, int32_t i, int32_t j,
                                          int32_t *members, int32_t cap, int32_t *len,
                                          int32_t *removal_depth) {
    if (!sk || !len) return fail(BNS_E_INVALID_ARG, "NULL argument");
    if (i < 0 || j < 0 || i >= sk->n || j >= sk->n || i == j) return fail(BNS_E_INVALID_ARG, "bad pair");
    if (cap < 0 || (cap > 0 && !members)) return fail(BNS_E_INVALID_ARG, "bad members buffer");
    sk->expand();
    const int64_t ij = (int64_t)i * sk->n + j;
    const int32_t d = sk->depth[ij];
    if (removal_depth) *removal_depth = d;
    if (d < 0) {
        *len = -1;
        return BNS_OK;
    }
    *len = d;
    const int64_t off = sk->sepoff[ij];
    for (int32_t k = 0; k < d && k < cap; ++k) members[k] = sk->pool[off + k];
    return BNS_OK;
}

extern "C" bns_status bns_skeleton_removals(const bns_skeleton *sk, int32_t *depth, int64_t *sep_off,
                                            int32_t *pool, int64_t pool_cap, int64_t *pool_len) {
    if (!sk) return fail(BNS_E_INVALID_ARG, "NULL skeleton");
    if (pool_cap < 0 || (pool_cap > 0 && !pool)) return fail(BNS_E_INVALID_ARG, "bad pool buffer");
    sk->expand();
    if (depth) std::memcpy(depth, sk->depth.data(), sk->depth.size() * sizeof(int32_t));
    if (sep_off) std::memcpy(sep_off, sk->sepoff.data(), sk->sepoff.size() * sizeof(int64_t));
    if (pool) std::memcpy(pool, sk->pool.data(), sizeof(int32_t) * (size_t)std::min<int64_t>(pool_cap, (int64_t)sk->pool.size()));
    if (pool_len) *pool_len = (int64_t)sk->pool.size();
    return BNS_OK;
}

extern "C" bns_status bns_skeleton_stats(const bns_skeleton *sk, bns_depth_stats *out, int32_t cap,
                                         int32_t *n_depths) {
    if (!sk || !n_depths) return fail(BNS_E_INVALID_ARG, "NULL argument");
    if (cap < 0 || (cap > 0 && !out)) return fail(BNS_E_INVALID_ARG, "bad stats buffer");
    *n_depths = (int32_t)sk->stats.size();
    for (int32_t d = 0; d < cap && d < (int32_t)sk->stats.size(); ++d) out[d] = sk->stats[d];
    return BNS_OK;
}

extern "C" void bns_skeleton_free(bns_skeleton *sk) { delete sk; }

// ---------------------------------------------------------------------------
// Batched form: device-resident queue, one persistent test launch per depth.
// ---------------------------------------------------------------------------
static void build_binom(int rows, std::vector<uint64_t> &B) {
    const uint64_t sat = ~0ull >> 2;
    B.assign((size_t)rows * kBinomK, 0);
    for (int n = 0; n < rows; ++n) {
        B[(size_t)n * kBinomK] = 1;
        for (int k = 1; k < kBinomK && k <= n; ++k) {
            const uint64_t a = B[(size_t)(n - 1) * kBinomK + k - 1];
            const uint64_t b = (k <= n - 1) ? B[(size_t)(n - 1) * kBinomK + k] : 0;
            B[(size_t)n * kBinomK + k] = (a >= sat || b >= sat || a + b >= sat) ? sat : a + b;
        }
    }
}

static bns_status dev_error(int32_t e) {
    switch (e) {
        case kDevTableTooLarge: return fail(BNS_E_TABLE_TOO_LARGE, "a test's contingency table exceeds the supported size");
        case kDevTooManyTests: return fail(BNS_E_TABLE_TOO_LARGE, "an edge has more conditioning sets than supported");
        case kDevDepthTooLarge: return fail(BNS_E_TABLE_TOO_LARGE, "the search exceeds the supported depth");
        case kDevUnitMismatch: return fail(BNS_E_INTERNAL, "test kernel instance and work units disagree");
        default: return fail(BNS_E_INTERNAL, "device error %d", e);
    }
}

static const int kDepthsPerLaunch = 8;
// Verification log entries (executed tests of one search) at most.
static const int64_t kErrLogEntries = 8 << 20;
// Split depths: merge tables (words) shared by a depth's tickets, the largest
// ticket count that is split, and default chunk / occupancy targets.
static const int64_t kSplitWords = 8 << 20;
static const int64_t kSplitTickets = 32768;
static const int32_t kSplitMinDefault = 4096;
static const int32_t kUnitsPerGroupDefault = 1;
// Column bytes of a search above which the test kernel deals tickets to its
// grab counters in runs (a quarter of MI355X's 256 MB last-level cache).
static const double kGrabRunBytes = 64.0 * 1024 * 1024;
// Results downloaded with the control block after each launch when they fit.
static const size_t kSpecBytes = 4u << 20;
static const size_t kSpecPoolWords = 64u << 10;

// Captures (once per distinct argument set) K consecutive depth sequences as
// one executable graph; the depth index lives in the device control block, so
// the same graph serves every starting depth.  Sequence tri_seq (if any) also
// holds the depth-1 contraction kernels, which act only when the device's
// depth is 1.
static bns_status depth_graph(DevCtx &dc, const DepthArgs &a, int grid, int K, bool init, int tri_seq,
                              uint32_t seq_units, hipStream_t s, GraphEntry **out) {
    for (size_t i = 0; i < dc.graphs.size(); ++i) {
        GraphEntry *g = dc.graphs[i].get();
        if (g->K == K && g->grid == grid && g->init == init && g->tri_seq == tri_seq && g->seq_units == seq_units &&
            std::memcmp(&g->args, &a, sizeof(a)) == 0) {
            // most recently used last: eviction takes the front
            std::rotate(dc.graphs.begin() + i, dc.graphs.begin() + i + 1, dc.graphs.end());
            *out = g;
            return BNS_OK;
        }
    }
    // the least recently used graph goes; its destructor waits for its last
    // replay (the host returns once the completion flag is up, before the
    // graph has ended)
    if (dc.graphs.size() >= 8) dc.graphs.erase(dc.graphs.begin());
    std::unique_ptr<GraphEntry> g(new GraphEntry());
    g->args = a;
    g->grid = grid;
    g->K = K;
    g->init = init;
    g->tri_seq = tri_seq;
    g->seq_units = seq_units;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t e = init ? launch_init_search(a, s) : hipSuccess;
    for (int i = 0; i < K && e == hipSuccess; ++i) {
        e = launch_depth_prepare(a, s);
        if (e == hipSuccess && i == tri_seq) e = launch_depth1_gram(a, s);
        if (e == hipSuccess)
            e = (init && i == 0 && a.pairs.part) ? launch_depth0_pairs(a, s)
                                                  : launch_depth_tests(a, grid, s, nullptr, nullptr,
                                                                       (int)((seq_units >> (2 * i)) & 3u));
        if (e == hipSuccess) e = launch_depth_apply(a, s);
    }
    if (e == hipSuccess) e = launch_publish(a, s);
    hipError_t e2 = hipStreamEndCapture(s, &g->graph);
    HIP_TRY(e);
    HIP_TRY(e2);
    HIP_TRY(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    HIP_TRY(hipEventCreateWithFlags(&g->done, hipEventDisableTiming));
    *out = g.get();
    dc.graphs.push_back(std::move(g));
    return BNS_OK;
}

// Waits for a launch's results: polls the completion flag that its last
// kernel writes into pinned memory (the stream itself reports completion
// ~14 us after that kernel ends), checking the stream now and then for
// errors; after 2 ms it blocks on the stream instead.  A stream that went
// idle without raising the flag is an internal error.
static hipError_t wait_published(hipStream_t s, const volatile unsigned long long *flag,
                                 unsigned long long want) {
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned it = 1;; ++it) {
        if (*flag == want) return hipSuccess;
        if ((it & 63u) != 0u) continue;
        hipError_t e = hipStreamQuery(s);
        if (e == hipErrorNotReady && std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(2000))
            e = hipStreamSynchronize(s);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return e;
        return *flag == want ? hipSuccess : hipErrorUnknown;
    }
}

static bns_status run_batched(DevCtx &dc, const bns_dataset *const *ds, int32_t P,
                              const double *alpha, const int32_t *maxd, const bns_options &o,
                              std::vector<bns_skeleton *> &outs) {
    Tile tile;
    if (!dc.search_lds) dc.search_lds = depth_tests_fit_lds(dc.lds_per_cu);
    bns_status st = make_tile(dc, o, &tile, true);
    if (st != BNS_OK) return st;
    hipStream_t s = o.stream ? (hipStream_t)o.stream : dc.stream;

    std::vector<ProbDev> probs((size_t)P);
    std::vector<int32_t> var2prob;
    std::vector<uint8_t> gcards;
    int64_t adj_total = 0, pairs_total = 0, m_max = 1, bit_total = 0;
    double col_bytes = 0.0;  // bytes of all columns
    int32_t G = 0, nmax = 0, dmax = -1;
    bool unbounded = false;
    for (int32_t k = 0; k < P; ++k) {
        const bns_dataset *d = ds[k];
        probs[k] = {d->d_data, d->ld, d->m, d->n, G, adj_total, alpha[k], maxd[k],
                    (int32_t)std::min<int64_t>(bit_total, INT32_MAX)};
        bit_total += (int64_t)d->n * ((d->n + 63) / 64);
        for (int32_t v = 0; v < d->n; ++v) var2prob.push_back(k);
        gcards.insert(gcards.end(), d->cards.begin(), d->cards.end());
        G += d->n;
        col_bytes += (double)d->n * (double)d->m;
        adj_total += (int64_t)d->n * d->n;
        pairs_total += (int64_t)d->n * (d->n - 1) / 2;
        nmax = std::max(nmax, d->n);
        m_max = std::max(m_max, d->m);
        if (maxd[k] < 0) unbounded = true;
        dmax = std::max(dmax, maxd[k]);
    }
    // binomial table (rebuilt only when a search needs more rows)
    const int brows = nmax + 1;
    if ((int)(dc.binom_host.size() / kBinomK) < brows) build_binom(brows, dc.binom_host);
    const std::vector<uint64_t> &Bfull = dc.binom_host;
    struct BView {
        const uint64_t *p;
        size_t n;
        size_t size() const { return n; }
        const uint64_t *data() const { return p; }
    } B{Bfull.data(), (size_t)brows * kBinomK};

    // One packed upload: problems, variable -> problem map, cardinalities,
    // binomial table (8-byte aligned sections).
    auto al8 = [](size_t x) { return (x + 7) & ~(size_t)7; };
    const size_t o_probs = 0;
    const size_t o_binom = al8(o_probs + sizeof(ProbDev) * (size_t)P);
    const size_t o_v2p = al8(o_binom + sizeof(uint64_t) * B.size());
    const size_t o_cards = al8(o_v2p + sizeof(int32_t) * (size_t)G);
    const bool per_prob = P > 1;
    const bool verify = o.report_errors != 0 && o.precision == BNS_PREC_FP32_RECHECK;
    // Depth 0 through the pair contraction (verification mode keeps the test
    // kernel, whose FP32 statistic it compares with FP64).
    PairPlan pp;
    if (!verify && o.depth0 == BNS_DEPTH0_PAIRS) {
        st = plan_pairs(dc, ds, P, pp);
        if (st != BNS_OK) return st;
    } else if (!verify && o.depth0 == BNS_DEPTH0_AUTO) {
        // the contraction's fixed cost (three launches, latency-bound
        // steps) pays once the depth's counting work is large
        double work = 0.0;
        for (int32_t k = 0; k < P; ++k) work += 0.5 * (double)ds[k]->n * (ds[k]->n - 1) * (double)ds[k]->m;
        if (work >= kPairsAutoWork && plan_pairs(dc, ds, P, pp) != BNS_OK) pp = PairPlan();
    }
    // Depth 1 through the masked Gram contractions (batched form; verification
    // mode keeps the test kernel, as at depth 0).
    bool tri_on = false;
    int64_t tri_cap = 0;
    int tri_target = 0, tri_grid = 0;
    // The automatic choice is the test kernel: the contraction evaluates every
    // depth-1 test, where the sequential order stops each edge at its first
    // accepting one (3x to 10x fewer tests on the measured workloads), and
    // each tile streams its variables' columns again (1,000 variables x
    // 200,000 samples: 4.0 M tests and 103 GB of column reads against 0.38 M
    // tests in the test kernel).
    if (!verify && o.form == BNS_FORM_BATCHED && (unbounded || dmax >= 1) && o.depth1 == BNS_DEPTH1_GRAM) {
        bool cards_ok = true;
        for (int32_t k = 0; k < P; ++k)
            for (uint8_t cv : ds[k]->cards) cards_ok = cards_ok && cv >= kTriMinCard && cv <= kTriMaxCard;
        tri_on = cards_ok;
        if (tri_on) {
            const int occ = tri_max_wg_per_cu();
            tri_target = 2 * dc.num_cu * occ;
            tri_grid = dc.num_cu * occ;
            // items if every node kept all its neighbours, plus room for the
            // sample chunks of small plans
            int64_t base_ub = 0;
            for (int32_t k = 0; k < P; ++k) {
                int64_t Rtot = 0;
                for (uint8_t cv : ds[k]->cards) Rtot += cv;
                for (uint8_t cv : ds[k]->cards) {
                    const int64_t nb = (Rtot - cv + 63) / 64;
                    base_ub += nb * (nb + 1) / 2 * ((cv + kTriCats - 1) / kTriCats);
                }
            }
            tri_cap = std::min<int64_t>(kTriItemsMax, (int64_t)tri_target + 2 * base_ub);
        }
    }
    const double tri_bytes = tri_on ? (double)sizeof(TriNode) * G + 8.0 * (double)adj_total +
                                          (double)tri_cap * kTriCats * 64 * 64 * 4
                                    : 0.0;
    const size_t o_gp = al8(o_cards + (size_t)G);
    const size_t o_ohvar = al8(o_gp + sizeof(GramProb) * pp.gps.size());
    const size_t o_ohcat = al8(o_ohvar + sizeof(int32_t) * pp.oh_var.size());
    const size_t o_varoh = al8(o_ohcat + sizeof(uint16_t) * pp.oh_cat.size());
    const size_t setup_bytes = al8(o_varoh + sizeof(int32_t) * pp.var_oh.size());
    const int64_t err_cap = verify ? kErrLogEntries : 0;
    const size_t rbytes = ((size_t)adj_total + 7) & ~(size_t)7;  // removal depths, padded for 8-byte copies
    {
        // every workspace buffer of the search (removal records: the first
        // launch's share; later growth is checked when it happens)
        const double bits = 8.0 * (double)std::min<int64_t>(std::max<int64_t>(bit_total, 1), kSmallBitWords);
        const double need = (double)setup_bytes + 9.0 * (double)adj_total + bits + (double)rbytes +
                            16.0 * G + (2.0 * sizeof(EdgeRec) + 8.0) * (double)pairs_total + sizeof(Ctl) +
                            4.0 * (double)kSplitWords + 4.0 * (double)kSplitTickets +
                            4.0 * 1024 + (per_prob ? sizeof(PStatDev) * (double)P * kMaxDepths + 8.0 * pairs_total : 0.0) +
                            8.0 * (double)err_cap + (double)(pp.part_bytes + pp.gram_bytes) + tri_bytes;
        st = check_workspace(o, need, "the skeleton search");
        if (st != BNS_OK) return st;
    }
    HIP_TRY(dc.setup.ensure(setup_bytes));
    HIP_TRY(dc.pinned(setup_bytes));
    {
        char *h = (char *)dc.hpin;
        std::memcpy(h + o_probs, probs.data(), sizeof(ProbDev) * (size_t)P);
        std::memcpy(h + o_binom, B.data(), sizeof(uint64_t) * B.size());
        std::memcpy(h + o_v2p, var2prob.data(), sizeof(int32_t) * (size_t)G);
        std::memcpy(h + o_cards, gcards.data(), (size_t)G);
        if (pp.on) {
            std::memcpy(h + o_gp, pp.gps.data(), sizeof(GramProb) * pp.gps.size());
            std::memcpy(h + o_ohvar, pp.oh_var.data(), sizeof(int32_t) * pp.oh_var.size());
            std::memcpy(h + o_ohcat, pp.oh_cat.data(), sizeof(uint16_t) * pp.oh_cat.size());
            std::memcpy(h + o_varoh, pp.var_oh.data(), sizeof(int32_t) * pp.var_oh.size());
        }
    }
    if (!(dc.setup_last_dev == dc.setup.p && dc.setup_last.size() == setup_bytes &&
          std::memcmp(dc.setup_last.data(), dc.hpin, setup_bytes) == 0)) {
        dc.setup_last_dev = nullptr;
        HIP_TRY(hipMemcpyAsync(dc.setup.p, dc.hpin, setup_bytes, hipMemcpyHostToDevice, s));
        dc.setup_last.assign((const char *)dc.hpin, (const char *)dc.hpin + setup_bytes);
        dc.setup_last_dev = dc.setup.p;
    }
    HIP_TRY(dc.adj.ensure((size_t)adj_total));
    HIP_TRY(dc.nbr.ensure(sizeof(int32_t) * (size_t)adj_total));
    HIP_TRY(dc.ipos.ensure(sizeof(int32_t) * (size_t)adj_total));
    // bit rows are used only by small searches (at most kSmallBitWords words)
    HIP_TRY(dc.adjbits.ensure(sizeof(uint64_t) * (size_t)std::min<int64_t>(std::max<int64_t>(bit_total, 1), kSmallBitWords)));
    HIP_TRY(dc.rdepth.ensure(rbytes));
    HIP_TRY(dc.deg.ensure(sizeof(int32_t) * (size_t)G));
    HIP_TRY(dc.rowcnt.ensure(sizeof(int32_t) * (size_t)G));
    HIP_TRY(dc.rowbase.ensure(sizeof(int64_t) * (size_t)G));
    HIP_TRY(dc.edges_tmp.ensure(sizeof(EdgeRec) * (size_t)pairs_total));
    HIP_TRY(dc.edges.ensure(sizeof(EdgeRec) * (size_t)pairs_total));
    HIP_TRY(dc.min_accept.ensure(sizeof(unsigned long long) * (size_t)pairs_total));
    HIP_TRY(dc.ctl.ensure(sizeof(Ctl)));
    HIP_TRY(dc.pool.ensure(sizeof(int32_t) * 1024));
    if (verify) {
        HIP_TRY(dc.err_val.ensure(sizeof(float) * (size_t)err_cap));
        HIP_TRY(dc.err_tag.ensure(sizeof(uint32_t) * (size_t)err_cap));
        HIP_TRY(dc.err_cnt.ensure(sizeof(unsigned long long)));
    }
    HIP_TRY(dc.pstat.ensure(per_prob ? sizeof(PStatDev) * (size_t)P * kMaxDepths : 256));
    HIP_TRY(dc.ecnt.ensure(per_prob ? sizeof(uint32_t) * 2 * (size_t)pairs_total : 256));
    if (pp.on) HIP_TRY(dc.pair_part.ensure((size_t)(pp.part_bytes + pp.gram_bytes)));
    if (tri_on) {
        HIP_TRY(dc.tri_node.ensure(sizeof(TriNode) * (size_t)G));
        HIP_TRY(dc.tri_rowoff.ensure(sizeof(int32_t) * (size_t)adj_total));
        HIP_TRY(dc.tri_eidx.ensure(sizeof(int32_t) * (size_t)adj_total));
        HIP_TRY(dc.tri_part.ensure(sizeof(int32_t) * (size_t)tri_cap * kTriCats * 64 * 64));
    }
    if (!dc.split_tab.p || dc.split_dirty) {
        HIP_TRY(dc.split_tab.ensure(sizeof(uint32_t) * (size_t)kSplitWords));
        HIP_TRY(dc.split_cnt.ensure(sizeof(uint32_t) * (size_t)kSplitTickets));
        HIP_TRY(hipMemsetAsync(dc.split_tab.p, 0, dc.split_tab.bytes, s));
        HIP_TRY(hipMemsetAsync(dc.split_cnt.p, 0, dc.split_cnt.bytes, s));
        dc.split_dirty = false;
    }

    DepthArgs a;
    std::memset(&a, 0, sizeof(a));
    a.probs = (const ProbDev *)(dc.setup.as<char>() + o_probs);
    a.n_probs = P;
    a.n_globals = G;
    a.var2prob = (const int32_t *)(dc.setup.as<char>() + o_v2p);
    a.cards = (const uint8_t *)(dc.setup.as<char>() + o_cards);
    a.binom = (const uint64_t *)(dc.setup.as<char>() + o_binom);
    a.binom_rows = brows;
    a.pad = 0;
    a.adj = dc.adj.as<uint8_t>();
    a.nbr = dc.nbr.as<int32_t>();
    a.ipos = dc.ipos.as<int32_t>();
    a.adjbits = dc.adjbits.as<uint64_t>();
    a.bit_words = bit_total;
    a.deg = dc.deg.as<int32_t>();
    a.rowcnt = dc.rowcnt.as<int32_t>();
    a.rowbase = dc.rowbase.as<int64_t>();
    a.edges_tmp = dc.edges_tmp.as<EdgeRec>();
    a.edges = dc.edges.as<EdgeRec>();
    a.min_accept = dc.min_accept.as<unsigned long long>();
    a.pstat = dc.pstat.as<PStatDev>();
    a.ecnt = dc.ecnt.as<uint32_t>();
    a.per_prob = per_prob ? 1 : 0;
    if (verify) {
        a.err_val = dc.err_val.as<float>();
        a.err_tag = dc.err_tag.as<uint32_t>();
        a.err_cnt = dc.err_cnt.as<unsigned long long>();
        a.err_cap = err_cap;
    }
    a.rdepth = dc.rdepth.as<int8_t>();
    a.pool = dc.pool.as<int32_t>();
    a.ctl = dc.ctl.as<Ctl>();
    a.tile = tile;
    a.split_tab = dc.split_tab.as<uint32_t>();
    a.split_cnt = dc.split_cnt.as<uint32_t>();
    a.split_words = kSplitWords;
    a.split_tickets = kSplitTickets;
    a.m_max = m_max;
    a.split_min = o.split_min_samples == 0 ? kSplitMinDefault : o.split_min_samples;
    a.units_per_group = o.units_per_group == 0 ? kUnitsPerGroupDefault : o.units_per_group;
    a.mode_policy = o.test_group;
    a.wave_depths = o.wave_depths;
    a.block_depths = o.block_depths;
    a.round_width = o.round_tests;
    a.edge_form = o.form == BNS_FORM_EDGE ? 1 : 0;
    // depth 1 in (edge, level) units: doubling levels, batched form, not in
    // verification mode; automatic when the search's columns (all its
    // datasets') exceed a quarter of the last-level cache (their tests re-read
    // X and Y from DRAM: 1,000 variables x 200,000 samples ran depth 1 in 14.7
    // instead of 23.1 ms, the 64-dataset batch in 9.3 instead of 12.3 ms);
    // smaller searches keep one test per unit, whose rank-major order skips
    // more speculative tests (60 x 50,000: 204 against 143 us)
    const bool xy_want = o.group_tests == BNS_GROUP_EDGE || (o.group_tests == BNS_GROUP_AUTO && col_bytes > kGrabRunBytes);
    a.xy_policy = (xy_want && o.form == BNS_FORM_BATCHED && o.round_tests == 0 && !verify && (unbounded || dmax >= 1))
                      ? 1 : 0;
    a.grab_fixed = o.tickets_per_grab;
    // Columns beyond a quarter of the last-level cache: deal the tickets to
    // the grab counters in runs of 64 (edges that share a column run on one
    // XCD); else one at a time.
    const bool runs = o.ticket_runs == 2 || (o.ticket_runs == 0 && col_bytes > kGrabRunBytes);
    a.grab_block_log2 = runs ? kGrabRunLog2 : 0;
    if (pp.on) {
        char *sb = dc.setup.as<char>();
        a.pairs.gp = (const GramProb *)(sb + o_gp);
        a.pairs.oh_var = (const int32_t *)(sb + o_ohvar);
        a.pairs.oh_cat = (const uint16_t *)(sb + o_ohcat);
        a.pairs.var_oh = (const int32_t *)(sb + o_varoh);
        a.pairs.part = dc.pair_part.as<int32_t>();
        a.pairs.gram = pp.gram_bytes ? a.pairs.part + pp.part_bytes / 4 : a.pairs.part;
        a.pairs.items = pp.items;
        a.pairs.tiles = pp.tiles;
        a.pairs.chunk = pp.chunk;
        a.pairs.T = pp.T;
        a.pairs.n_gp = P;
        a.pairs.gram_grid = (int)std::min<int64_t>(pp.items, (int64_t)dc.num_cu * gram_max_wg_per_cu(pp.T));
    }
    if (tri_on) {
        a.tri.node = dc.tri_node.as<TriNode>();
        a.tri.rowoff = dc.tri_rowoff.as<int32_t>();
        a.tri.eidx = dc.tri_eidx.as<int32_t>();
        a.tri.part = dc.tri_part.as<int32_t>();
        a.tri.part_items = tri_cap;
        a.tri.target_items = tri_target;
        a.tri.grid = tri_grid;
    }

    const int lds_bytes = tile.lds_words * 4;
    int wg = o.wg_per_cu ? o.wg_per_cu : depth_tests_max_wg_per_cu(lds_bytes);
    const int grid = std::max(1, dc.num_cu * wg);
    a.test_waves = grid * kWaves;
    a.n_pairs = pairs_total;
    a.edge_grid = (int)std::max<int64_t>(1, std::min<int64_t>(512, (pairs_total + kWG - 1) / kWG));

    // Timing: the depth sequences of a launch are enqueued directly, each test
    // kernel launched with a start/stop event pair, and synchronised once.
    struct EvGuard {
        std::vector<hipEvent_t> v;
        ~EvGuard() {
            for (hipEvent_t e : v) (void)hipEventDestroy(e);
        }
    } evg;
    if (o.timing) {
        evg.v.assign(2 * (size_t)kDepthsPerLaunch, nullptr);
        for (hipEvent_t &e : evg.v) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    }

    // Depths run in launches of up to kDepthsPerLaunch depth sequences; the
    // host reads the control block once per launch.  A depth with no tests
    // marks the search done and the kernels of any later sequence in the same
    // launch return at once.
    const bool use_graph = o.use_graph != 0 && !o.timing && !verify;
    GraphEntry *ge = nullptr;
    const int per_launch = (use_graph || o.timing) ? kDepthsPerLaunch : 1;
    std::vector<bns_depth_stats> stats;
    unsigned long long alive = (unsigned long long)pairs_total;  // edges alive at depth d
    unsigned long long pool_used = 0;
    bool spec = false;
    size_t spec_pool = 0;
    int d = 0;
    for (;;) {
        if (!unbounded && d > dmax) break;
        if (d >= kMaxDepths) return fail(BNS_E_TABLE_TOO_LARGE, "the search exceeds %d depths", kMaxDepths);
        int K = per_launch;
        // Searches on one device tend to repeat: the first launch covers as
        // many depth sequences as the last search needed (a depth sequence
        // of a finished search still launches its kernels).
        if (d == 0 && dc.last_sequences > 0) K = std::min(K, dc.last_sequences);
        if (!unbounded) K = std::min(K, dmax + 1 - d);
        K = std::min(K, kMaxDepths - d);
        // Sepset slots for every edge that may be removed in these depths.
        unsigned long long slots = 0;
        for (int i = 0; i < K; ++i)
            if (d + i > 0) slots += alive * (unsigned long long)(d + i + 3);
        const size_t need = (size_t)(pool_used + slots);
        if (need > dc.pool.bytes / sizeof(int32_t)) {
            st = check_workspace(o, 4.0 * (double)std::max(need, 2 * dc.pool.bytes / sizeof(int32_t)),
                                 "the skeleton search's removal records");
            if (st != BNS_OK) return st;
            DevBuf nb;
            HIP_TRY(nb.ensure(sizeof(int32_t) * std::max(need, 2 * dc.pool.bytes / sizeof(int32_t))));
            if (pool_used)
                HIP_TRY(hipMemcpyAsync(nb.p, dc.pool.p, sizeof(int32_t) * (size_t)pool_used, hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
            std::swap(dc.pool.p, nb.p);
            std::swap(dc.pool.bytes, nb.bytes);
            a.pool = dc.pool.as<int32_t>();
        }
        // The last kernel of a launch writes the control block into pinned
        // host memory, and when the results are small (most searches finish
        // within one launch) the removal depths and the first removal records
        // too: one round trip, no copies.
        spec_pool = 0;
        spec = rbytes + sizeof(int32_t) * kSpecPoolWords <= kSpecBytes;
        if (spec) {
            spec_pool = std::min<size_t>(kSpecPoolWords, dc.pool.bytes / sizeof(int32_t));
            HIP_TRY(dc.results(rbytes + sizeof(int32_t) * spec_pool));
        }
        a.h_ctl = dc.h_ctl;
        a.h_res = spec ? (char *)dc.hres : nullptr;
        a.res_rbytes = (int64_t)rbytes;
        a.res_pool_words = (int64_t)spec_pool;
        a.pub_seq = (unsigned long long *)dc.pub;
        a.pub_cnt = (unsigned int *)((char *)dc.pub + 8);
        a.h_flag = dc.h_flag;
        // the sequence of this launch that holds depth 1, when it runs
        // through the contraction
        const int tri_seq = (tri_on && d <= 1 && 1 < d + K) ? 1 - d : -1;
        // the test kernel instance of each sequence (its depth's work units)
        uint32_t seq_units = 0;
        for (int i = 0; i < K; ++i) seq_units |= (uint32_t)depth_units(a, d + i) << (2 * i);
        if (use_graph) {
            st = depth_graph(dc, a, grid, K, d == 0, tri_seq, seq_units, s, &ge);
            if (st != BNS_OK) return st;
            HIP_TRY(hipGraphLaunch(ge->exec, s));
            HIP_TRY(hipEventRecord(ge->done, s));
        } else {
            if (d == 0) HIP_TRY(launch_init_search(a, s));
            for (int i = 0; i < K; ++i) {
                HIP_TRY(launch_depth_prepare(a, s));
                if (d == 0 && i == 0 && a.pairs.part) {
                    if (o.timing) HIP_TRY(hipEventRecord(evg.v[0], s));
                    HIP_TRY(launch_depth0_pairs(a, s));
                    if (o.timing) HIP_TRY(hipEventRecord(evg.v[1], s));
                } else if (i == tri_seq) {
                    if (o.timing) HIP_TRY(hipEventRecord(evg.v[2 * i], s));
                    HIP_TRY(launch_depth1_gram(a, s));
                    HIP_TRY(launch_depth_tests(a, grid, s, nullptr, nullptr, depth_units(a, d + i)));
                    if (o.timing) HIP_TRY(hipEventRecord(evg.v[2 * i + 1], s));
                } else if (o.timing) {
                    HIP_TRY(launch_depth_tests(a, grid, s, evg.v[2 * i], evg.v[2 * i + 1], depth_units(a, d + i)));
                } else {
                    HIP_TRY(launch_depth_tests(a, grid, s, nullptr, nullptr, depth_units(a, d + i)));
                }
                HIP_TRY(launch_depth_apply(a, s));
            }
            HIP_TRY(launch_publish(a, s));
        }
        {
            const hipError_t we = wait_published(s, dc.h_flag, ++dc.pub_expected);
            if (we != hipSuccess) {
                // re-synchronise the expected count with the device's
                unsigned long long v = 0;
                if (hipStreamSynchronize(s) == hipSuccess && hipMemcpy(&v, dc.pub, sizeof(v), hipMemcpyDeviceToHost) == hipSuccess)
                    dc.pub_expected = v;
                HIP_TRY(we);
            }
        }
        const Ctl &c = *dc.h_ctl;
        if (c.error) {
            dc.split_dirty = true;  // a depth may have stopped with partial merge tables
            return dev_error(c.error);
        }
        const int reached = c.depth;  // depths d .. reached-1 completed
        for (int dd = d; dd < reached; ++dd) {
            const DepthStatDev &sd = c.stats[dd];
            bns_depth_stats r;
            std::memset(&r, 0, sizeof(r));
            r.depth = dd;
            r.edges = (int64_t)sd.edges;
            r.tests_required = (int64_t)sd.required;
            r.tests_executed = (int64_t)sd.executed;
            r.removed = (int64_t)sd.removed;
            r.rechecks = (int64_t)sd.rechecks;
            r.tickets = (int64_t)sd.tickets;
            r.operand_bytes = sd.operand_bytes;
            r.test_group = sd.mode + 1;
            r.chunks = sd.chunks;
            r.chunk_samples = sd.chunk_len;
            if (sd.t_end && sd.t_start) {
                const unsigned long long t0 = sd.t_start;
                if (sd.t_end > t0) r.span_seconds = (double)(sd.t_end - t0) / (1e3 * dc.wall_khz);
            }
            if (o.timing) {
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, evg.v[2 * (dd - d)], evg.v[2 * (dd - d) + 1]));
                r.kernel_seconds = ms * 1e-3;
            }
            stats.push_back(r);
            alive = sd.edges - sd.removed;
        }
        pool_used = c.pool_used;
        if (c.done) {
            // sequences this search launched up to the one that found no test
            dc.last_sequences = reached + (small_search(a) ? 0 : 1);
            break;
        }
        if (reached != d + K) return fail(BNS_E_INTERNAL, "depth counter %d after launch from %d", reached, d);
        d = reached;
    }

    // Results: removal depths (int8 per pair; -1 = kept) and the removal
    // records of depth >= 1, unless the last round trip brought them.
    const size_t pbytes = sizeof(int32_t) * (size_t)pool_used;
    if (!(spec && pool_used <= spec_pool)) {
        HIP_TRY(dc.results(rbytes + pbytes));
        HIP_TRY(hipMemcpyAsync(dc.hres, dc.rdepth.p, (size_t)adj_total, hipMemcpyDeviceToHost, s));
        if (pool_used)
            HIP_TRY(hipMemcpyAsync((char *)dc.hres + rbytes, dc.pool.p, pbytes, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    // Verification log: relative FP32 errors by (problem, depth).
    std::vector<std::vector<std::vector<float>>> errv;
    std::vector<std::vector<int64_t>> errflip;
    if (verify) {
        unsigned long long cnt = 0;
        HIP_TRY(hipMemcpyAsync(&cnt, dc.err_cnt.p, sizeof(cnt), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if ((int64_t)cnt > err_cap)
            return fail(BNS_E_NOMEM, "verification log overflow: %llu tests, room for %lld", cnt, (long long)err_cap);
        std::vector<float> hv((size_t)cnt);
        std::vector<uint32_t> ht((size_t)cnt);
        if (cnt) {
            HIP_TRY(hipMemcpyAsync(hv.data(), dc.err_val.p, sizeof(float) * (size_t)cnt, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(ht.data(), dc.err_tag.p, sizeof(uint32_t) * (size_t)cnt, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
        errv.assign((size_t)P, std::vector<std::vector<float>>(kMaxDepths));
        errflip.assign((size_t)P, std::vector<int64_t>(kMaxDepths, 0));
        for (size_t i = 0; i < (size_t)cnt; ++i) {
            const uint32_t k = ht[i] >> 16, dd = ht[i] & 0xffu;
            if (k >= (uint32_t)P || dd >= (uint32_t)kMaxDepths) return fail(BNS_E_INTERNAL, "corrupt verification record");
            errv[k][dd].push_back(hv[i]);
            errflip[k][dd] += (ht[i] >> 8) & 1u;
        }
    }
    auto fill_err = [&](bns_depth_stats &r, int k, int dd) {
        if (!verify || dd >= kMaxDepths) return;
        std::vector<float> &v = errv[(size_t)k][(size_t)dd];
        r.err_tests = (int64_t)v.size();
        r.err_flips = errflip[(size_t)k][(size_t)dd];
        if (v.empty()) return;
        std::sort(v.begin(), v.end());
        // nearest-rank percentiles
        auto rank = [&](double q) {
            size_t i = (size_t)std::ceil(q * (double)v.size());
            return (double)v[std::min(v.size() - 1, i ? i - 1 : 0)];
        };
        r.err_max = (double)v.back();
        r.err_p50 = rank(0.5);
        r.err_p99 = rank(0.99);
    };
    // Per-problem counters of a multi-dataset search (small: P x 64 records).
    std::vector<PStatDev> hps;
    if (per_prob) {
        hps.resize((size_t)P * kMaxDepths);
        HIP_TRY(hipMemcpyAsync(hps.data(), dc.pstat.p, sizeof(PStatDev) * hps.size(), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    const char *hres = (const char *)dc.hres;
    const int8_t *hdep = (const int8_t *)hres;
    const int32_t *hpool = (const int32_t *)(hres + rbytes);
    std::vector<std::unique_ptr<bns_skeleton>> sks((size_t)P);
    for (int32_t k = 0; k < P; ++k) {
        sks[k].reset(new bns_skeleton());
        bns_skeleton *sk = sks[k].get();
        const int n = ds[k]->n;
        const int64_t base = probs[k].adj_off, nn = (int64_t)n * n;
        sk->n = n;
        sk->rdep.assign(hdep + base, hdep + base + nn);
        if (!per_prob) {
            sk->stats = stats;
            for (size_t dd = 0; dd < sk->stats.size(); ++dd) fill_err(sk->stats[dd], k, (int)dd);
            continue;
        }
        // This problem's own counters, up to its last depth with a test; the
        // launch timings (kernel_seconds, span_seconds) are the batch's.
        for (size_t dd = 0; dd < stats.size() && dd < (size_t)kMaxDepths; ++dd) {
            const PStatDev &ps = hps[(size_t)k * kMaxDepths + dd];
            if (ps.tickets == 0) break;
            bns_depth_stats r = stats[dd];
            r.edges = (int64_t)ps.edges;
            r.tickets = (int64_t)ps.tickets;
            r.tests_required = (int64_t)ps.required;
            r.tests_executed = (int64_t)ps.executed;
            r.removed = (int64_t)ps.removed;
            r.rechecks = (int64_t)ps.rechecks;
            r.operand_bytes = (double)ps.executed * (double)(dd + 2) * (double)ds[k]->m;
            fill_err(r, k, (int)dd);
            sk->stats.push_back(r);
        }
    }
    for (unsigned long long q = 0; q < pool_used;) {
        const int32_t k = hpool[q], i = hpool[q + 1], j = hpool[q + 2];
        if (k < 0 || k >= P) return fail(BNS_E_INTERNAL, "corrupt removal record");
        bns_skeleton *sk = sks[k].get();
        const int n = sk->n;
        if (i < 0 || j < 0 || i >= n || j >= n) return fail(BNS_E_INTERNAL, "corrupt removal record");
        const int32_t dd = sk->rdep[(size_t)((int64_t)i * n + j)];
        if (dd <= 0) return fail(BNS_E_INTERNAL, "removal record for a pair not removed at depth >= 1");
        sk->rec_pair.push_back((int64_t)i * n + j);
        sk->rec_off.push_back((int64_t)sk->pool.size());
        sk->pool.insert(sk->pool.end(), hpool + q + 3, hpool + q + 3 + dd);
        q += (unsigned long long)dd + 3;
    }
    for (int32_t k = 0; k < P; ++k) outs[k] = sks[k].release();
    return BNS_OK;
}

// ---------------------------------------------------------------------------
// Plain form: the host walks the tests in the sequential order; every test is
// one sample-parallel counting launch plus a finishing launch and a readback.
// ---------------------------------------------------------------------------
static bns_status plain_test(DevCtx &dc, const bns_dataset *ds, const Tile &tile, hipStream_t s,
                             const int32_t *vars, int ncols, double alpha, CiOutDev *res) {
    PlainTest pt;
    std::memset(&pt, 0, sizeof(pt));
    pt.ncols = ncols;
    int64_t T = 1, Z = 1;
    for (int k = 0; k < ncols; ++k) {
        pt.vars[k] = vars[k];
        T *= ds->cards[vars[k]];
        if (k >= 2) Z *= ds->cards[vars[k]];
        if (T > (int64_t)kMaxCells) return fail(BNS_E_TABLE_TOO_LARGE, "table exceeds %u cells", kMaxCells);
    }
    const int64_t spb = 4096;
    const int nblocks = (int)std::max<int64_t>(1, (ds->m + spb - 1) / spb);
    HIP_TRY(dc.plain_part.ensure(sizeof(uint32_t) * (size_t)T * (size_t)nblocks));
    const int64_t ws = T + (int64_t)(ds->cards[vars[0]] + ds->cards[vars[1]] + 1) * Z;
    HIP_TRY(dc.plain_ws.ensure(sizeof(uint32_t) * (size_t)ws));
    HIP_TRY(dc.plain_out.ensure(sizeof(CiOutDev)));
    HIP_TRY(launch_plain_count(ds->d_data, ds->ld, ds->m, ds->d_cards, pt, spb, nblocks,
                               dc.plain_part.as<uint32_t>(), T, tile.lds_words, s));
    HIP_TRY(launch_plain_finish(ds->d_cards, pt, nblocks, dc.plain_part.as<uint32_t>(), T,
                                dc.plain_ws.as<uint32_t>(), alpha, tile.stat, tile.df_rule,
                                dc.plain_out.as<CiOutDev>(), s));
    HIP_TRY(hipMemcpyAsync(dc.h_out, dc.plain_out.p, sizeof(CiOutDev), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *res = *dc.h_out;
    return BNS_OK;
}

static bool next_subset(std::vector<int32_t> &idx, int d, int p) {
    int k = d - 1;
    while (k >= 0 && idx[k] == p - d + k) --k;
    if (k < 0) return false;
    ++idx[k];
    for (int l = k + 1; l < d; ++l) idx[l] = idx[l - 1] + 1;
    return true;
}

static bns_status run_plain(DevCtx &dc, const bns_dataset *ds, double alpha, int32_t max_depth,
                            const bns_options &o, bns_skeleton **out) {
    Tile tile;
    bns_status st = make_tile(dc, o, &tile);
    if (st != BNS_OK) return st;
    hipStream_t s = o.stream ? (hipStream_t)o.stream : dc.stream;
    const int n = ds->n;
    std::unique_ptr<bns_skeleton> sk(new bns_skeleton());
    sk->full = true;
    sk->n = n;
    sk->adj.assign((size_t)n * n, 0);
    sk->depth.assign((size_t)n * n, -1);
    sk->sepoff.assign((size_t)n * n, -1);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) sk->adj[(size_t)i * n + j] = (i != j);
    std::vector<std::vector<int32_t>> a((size_t)n);
    std::vector<int32_t> vars(kMaxCols), candA, candB, idx;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (o.timing) {
        HIP_TRY(hipEventCreate(&ev0));
        HIP_TRY(hipEventCreate(&ev1));
    }
    for (int d = 0; max_depth < 0 || d <= max_depth; ++d) {
        if (d >= kMaxDepths) return fail(BNS_E_TABLE_TOO_LARGE, "the search exceeds %d depths", kMaxDepths);
        for (int v = 0; v < n; ++v) {
            a[v].clear();
            for (int u = 0; u < n; ++u)
                if (sk->adj[(size_t)v * n + u]) a[v].push_back(u);
        }
        bool any = false;
        for (int i = 0; i < n && !any; ++i)
            for (int j = i + 1; j < n; ++j)
                if (sk->adj[(size_t)i * n + j] && (d == 0 || (int)a[i].size() - 1 >= d || (int)a[j].size() - 1 >= d)) {
                    any = true;
                    break;
                }
        if (!any) break;
        if (d > kMaxZ) return fail(BNS_E_TABLE_TOO_LARGE, "the search exceeds depth %d", kMaxZ);
        bns_depth_stats r;
        std::memset(&r, 0, sizeof(r));
        r.depth = d;
        if (o.timing) HIP_TRY(hipEventRecord(ev0, s));
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                if (!sk->adj[(size_t)i * n + j]) continue;
                ++r.edges;
                vars[0] = i;
                vars[1] = j;
                bool removed = false;
                for (int side = 0; side < 2 && !removed; ++side) {
                    if (d == 0 && side == 1) break;
                    std::vector<int32_t> &cand = side == 0 ? candA : candB;
                    cand.clear();
                    const int owner = side == 0 ? i : j, other = side == 0 ? j : i;
                    for (int u : a[owner])
                        if (u != other) cand.push_back(u);
                    const int p = (int)cand.size();
                    if (p < d) continue;
                    idx.resize((size_t)d);
                    for (int k = 0; k < d; ++k) idx[k] = k;
                    do {
                        for (int k = 0; k < d; ++k) vars[2 + k] = cand[idx[k]];
                        CiOutDev res;
                        st = plain_test(dc, ds, tile, s, vars.data(), d + 2, alpha, &res);
                        if (st != BNS_OK) return st;
                        ++r.tests_required;
                        ++r.tests_executed;
                        r.operand_bytes += (double)(d + 2) * (double)ds->m;
                        if (res.p > alpha) {
                            const size_t ij = (size_t)i * n + j, ji = (size_t)j * n + i;
                            sk->adj[ij] = sk->adj[ji] = 0;
                            sk->depth[ij] = sk->depth[ji] = d;
                            sk->sepoff[ij] = sk->sepoff[ji] = (int64_t)sk->pool.size();
                            for (int k = 0; k < d; ++k) sk->pool.push_back(vars[2 + k]);
                            ++r.removed;
                            removed = true;
                            break;
                        }
                    } while (d > 0 && next_subset(idx, d, p));
                }
            }
        if (o.timing) {
            HIP_TRY(hipEventRecord(ev1, s));
            HIP_TRY(hipEventSynchronize(ev1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1));
            r.kernel_seconds = ms * 1e-3;
        }
        sk->stats.push_back(r);
    }
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    *out = sk.release();
    return BNS_OK;
}

// ---------------------------------------------------------------------------
// Skeleton entry points
// ---------------------------------------------------------------------------
extern "C" bns_status bns_pc_skeleton_batch(const bns_dataset *const *ds, int32_t n_problems,
                                            const double *alpha, const int32_t *max_depth,
                                            const bns_options *opt, bns_skeleton **outs) {
    if (!ds || !alpha || !max_depth || !outs || n_problems < 1)
        return fail(BNS_E_INVALID_ARG, "NULL argument or n_problems < 1");
    for (int32_t k = 0; k < n_problems; ++k) outs[k] = nullptr;
    bns_options o;
    bns_status st = read_options(opt, &o);
    if (st != BNS_OK) return st;
    int64_t pairs = 0;
    for (int32_t k = 0; k < n_problems; ++k) {
        if (!ds[k]) return fail(BNS_E_INVALID_ARG, "dataset %d is NULL", k);
        if (!(alpha[k] > 0.0 && alpha[k] < 1.0)) return fail(BNS_E_INVALID_ARG, "alpha[%d] must be in (0, 1)", k);
        if (max_depth[k] < -1) return fail(BNS_E_INVALID_ARG, "max_depth[%d] must be >= -1", k);
        if (ds[k]->device != ds[0]->device) return fail(BNS_E_INVALID_ARG, "datasets on different devices");
        pairs += (int64_t)ds[k]->n * (ds[k]->n - 1) / 2;
    }
    if (pairs > (int64_t)UINT32_MAX) return fail(BNS_E_INVALID_ARG, "too many variable pairs in one batch");
    if (o.form == BNS_FORM_PLAIN && n_problems != 1)
        return fail(BNS_E_INVALID_ARG, "the plain form runs one dataset at a time");
    DevCtx *dc = nullptr;
    st = get_ctx(ds[0]->device, &dc);
    if (st != BNS_OK) return st;
    DeviceGuard dg(ds[0]->device);
    if (!dg.ok) return fail(BNS_E_DEVICE, "cannot select device %d", ds[0]->device);
    std::lock_guard<std::mutex> lk(dc->mu);
    if (o.form == BNS_FORM_PLAIN) return run_plain(*dc, ds[0], alpha[0], max_depth[0], o, outs);
    std::vector<bns_skeleton *> res((size_t)n_problems, nullptr);
    st = run_batched(*dc, ds, n_problems, alpha, max_depth, o, res);
    if (st != BNS_OK) {
        for (auto *r : res) delete r;
        return st;
    }
    for (int32_t k = 0; k < n_problems; ++k) outs[k] = res[k];
    return BNS_OK;
}

// ---------------------------------------------------------------------------
// Autotuning of the batched search's launch options
// ---------------------------------------------------------------------------
struct TuneEntry {
    std::string device;  // architecture and compute units
    std::vector<int64_t> key;
    bns_options best;
};
static std::mutex g_tune_mu;
static std::vector<TuneEntry> g_tune;
static bool g_tune_loaded = false;

// The tuned options that are kept (stream excluded), in file order.
static const int kTuneFields = 12;
static int32_t *tune_field(bns_options &o, int i) {
    int32_t *f[] = {&o.test_group, &o.max_replicas, &o.lds_bytes, &o.tickets_per_grab, &o.split_min_samples,
                    &o.units_per_group, &o.depth0, &o.round_tests, (int32_t *)&o.wave_depths,
                    (int32_t *)&o.block_depths, &o.depth1, &o.group_tests};
    return i < kTuneFields ? f[i] : nullptr;
}

// Persistent cache of tuned options: the file named by BNS_TUNE_CACHE, else
// $XDG_CACHE_HOME/bns_autotune.txt, else $HOME/.cache/bns_autotune.txt (no
// file when none is set).  One line per entry:
//   bns4 <device> <key, comma-separated> <twelve option values>
// Unreadable or malformed lines are ignored; the file is only a shortcut
// (options never change results).
static std::string tune_path() {
    if (const char *p = std::getenv("BNS_TUNE_CACHE")) return p;
    if (const char *x = std::getenv("XDG_CACHE_HOME")) return std::string(x) + "/bns_autotune.txt";
    if (const char *h = std::getenv("HOME")) return std::string(h) + "/.cache/bns_autotune.txt";
    return "";
}

static void tune_load_file() {
    g_tune_loaded = true;
    const std::string path = tune_path();
    if (path.empty()) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream in(line);
        std::string tag, dev, keys;
        if (!(in >> tag >> dev >> keys) || tag != "bns4") continue;
        TuneEntry e;
        e.device = dev;
        bool ok = true;
        std::istringstream ks(keys);
        for (std::string tok; ok && std::getline(ks, tok, ',');) {
            char *end = nullptr;
            e.key.push_back(std::strtoll(tok.c_str(), &end, 10));
            ok = !tok.empty() && *end == '\0';
        }
        bns_options_default(&e.best);
        for (int i = 0; i < kTuneFields && ok; ++i) {
            long long v = 0;
            if (!(in >> v)) ok = false;
            else *tune_field(e.best, i) = (int32_t)v;
        }
        bns_options checked;
        if (ok && read_options(&e.best, &checked) == BNS_OK) g_tune.push_back(e);
    }
}

static void tune_save_entry(const TuneEntry &e) {
    const std::string path = tune_path();
    if (path.empty()) return;
    FILE *f = std::fopen(path.c_str(), "a");
    if (!f) return;  // a cache that cannot be written is not an error
    std::fprintf(f, "bns4 %s ", e.device.c_str());
    for (size_t i = 0; i < e.key.size(); ++i) std::fprintf(f, "%s%lld", i ? "," : "", (long long)e.key[i]);
    bns_options o = e.best;
    for (int i = 0; i < kTuneFields; ++i) std::fprintf(f, " %d", *tune_field(o, i));
    std::fprintf(f, "\n");
    std::fclose(f);
}

extern "C" bns_status bns_autotune(const bns_dataset *const *ds, int32_t n_problems,
                                   const double *alpha, const int32_t *max_depth,
                                   const bns_options *base, int32_t trials, bns_options *best) {
    if (!ds || !alpha || !max_depth || !best || n_problems < 1)
        return fail(BNS_E_INVALID_ARG, "NULL argument or n_problems < 1");
    if (trials < 0 || trials > 100) return fail(BNS_E_INVALID_ARG, "trials must be in [0, 100]");
    bns_options o;
    bns_status st = read_options(base, &o);
    if (st != BNS_OK) return st;
    if (o.form != BNS_FORM_BATCHED) return fail(BNS_E_INVALID_ARG, "autotuning applies to the batched form");
    for (int32_t k = 0; k < n_problems; ++k)
        if (!ds[k]) return fail(BNS_E_INVALID_ARG, "dataset %d is NULL", k);
    const int reps = trials ? trials : 5;
    // workload key: sizes, alphas (bits), depths, precision
    std::vector<int64_t> key;
    key.push_back(o.precision);
    for (int32_t k = 0; k < n_problems; ++k) {
        int64_t ab;
        std::memcpy(&ab, &alpha[k], sizeof(ab));
        key.insert(key.end(), {ds[k]->n, ds[k]->m, ab, max_depth[k]});
    }
    std::string device;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, ds[0]->device) != hipSuccess)
            return fail(BNS_E_DEVICE, "cannot read the properties of device %d", ds[0]->device);
        char buf[160];
        std::snprintf(buf, sizeof(buf), "%s/%dcu", prop.gcnArchName, prop.multiProcessorCount);
        for (char *c = buf; *c; ++c)
            if (*c == ' ') *c = '_';
        device = buf;
    }
    // options that base fixes are part of the key
    for (int i = 0; i < kTuneFields; ++i) key.push_back(*tune_field(o, i));
    key.push_back(o.statistic);
    key.push_back(o.df_rule);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (!g_tune_loaded) tune_load_file();
        for (const TuneEntry &e : g_tune)
            if (e.device == device && e.key == key) {
                *best = o;
                for (int i = 0; i < kTuneFields; ++i) *tune_field(*best, i) = *tune_field(const_cast<bns_options &>(e.best), i);
                best->stream = o.stream;
                return BNS_OK;
            }
    }
    std::vector<bns_skeleton *> outs((size_t)n_problems, nullptr);
    auto timed = [&](const bns_options &c, double *sec) -> bns_status {
        std::vector<double> t;
        for (int r = 0; r < reps + 1; ++r) {  // first run warms caches and graphs
            const auto t0 = std::chrono::steady_clock::now();
            bns_status s2 = bns_pc_skeleton_batch(ds, n_problems, alpha, max_depth, &c, outs.data());
            const auto t1 = std::chrono::steady_clock::now();
            for (auto *h : outs) bns_skeleton_free(h);
            if (s2 != BNS_OK) return s2;
            if (r > 0) t.push_back(std::chrono::duration<double>(t1 - t0).count());
        }
        std::sort(t.begin(), t.end());
        *sec = t[t.size() / 2];
        return BNS_OK;
    };
    bns_options cur = o;
    double cur_t = 0.0;
    st = timed(cur, &cur_t);
    if (st != BNS_OK) return st;
    // Per depth: one wave or one workgroup per test, whichever ran that
    // depth's test kernel in less time (device-clock spans).  The skeleton,
    // and so each depth's edges and tests, is the same either way.
    auto depth_spans = [&](const bns_options &c, std::vector<double> *med) -> bns_status {
        std::vector<std::vector<double>> sp;
        for (int r = 0; r < reps + 1; ++r) {
            bns_status s2 = bns_pc_skeleton_batch(ds, n_problems, alpha, max_depth, &c, outs.data());
            if (s2 == BNS_OK && r > 0) {
                const std::vector<bns_depth_stats> &dst = outs[0]->stats;
                if (sp.size() < dst.size()) sp.resize(dst.size());
                for (size_t d = 0; d < dst.size(); ++d) sp[d].push_back(dst[d].span_seconds);
            }
            for (auto *h : outs) bns_skeleton_free(h);
            if (s2 != BNS_OK) return s2;
        }
        med->clear();
        for (std::vector<double> &v : sp) {
            std::sort(v.begin(), v.end());
            med->push_back(v.empty() ? 0.0 : v[v.size() / 2]);
        }
        return BNS_OK;
    };
    // The per-depth choice under cur's other options, kept when the whole
    // search gets faster.
    auto try_depths = [&]() -> bns_status {
        if (o.test_group != 0 || o.wave_depths != 0u || o.block_depths != 0u) return BNS_OK;
        bns_options cw = cur, cb = cur, cm = cur;
        cw.wave_depths = cw.block_depths = cb.wave_depths = cb.block_depths = 0u;
        cw.test_group = 1;
        cb.test_group = 2;
        std::vector<double> sw, sb;
        bns_status s2 = depth_spans(cw, &sw);
        if (s2 != BNS_OK) return s2;
        s2 = depth_spans(cb, &sb);
        if (s2 != BNS_OK) return s2;
        cm.test_group = 0;
        cm.wave_depths = cm.block_depths = 0u;
        for (size_t d = 0; d < std::min(sw.size(), sb.size()) && d < 32; ++d)
            (sw[d] < sb[d] ? cm.wave_depths : cm.block_depths) |= 1u << d;
        if (std::memcmp(&cm, &cur, sizeof(cm)) == 0) return BNS_OK;
        double t = 0.0;
        s2 = timed(cm, &t);
        if (s2 != BNS_OK) return s2;
        if (t < cur_t * 0.99) {
            cur = cm;
            cur_t = t;
        }
        return BNS_OK;
    };
    // Groups per depth first (they matter most); then every combination of
    // replication cap, LDS budget and grab size that base leaves open (a grid
    // of at most 27, so the result does not depend on the order of a greedy
    // descent), keeping a combination only on a clear gain; then the groups
    // per depth again under the chosen options.
    st = try_depths();
    if (st != BNS_OK) return st;
    const int32_t reps_opts[] = {0, 16, 64};
    const int32_t lds_opts[] = {0, 32768, 49152};
    const int32_t grab_opts[] = {0, 1, 2};
    const bns_options start = cur;
    for (int ir = 0; ir < 3; ++ir) {
        if (o.max_replicas && ir) break;
        for (int il = 0; il < 3; ++il) {
            if (o.lds_bytes && il) break;
            for (int ig = 0; ig < 3; ++ig) {
                if (o.tickets_per_grab && ig) break;
                bns_options c = start;
                if (!o.max_replicas) c.max_replicas = reps_opts[ir];
                if (!o.lds_bytes) c.lds_bytes = lds_opts[il];
                if (!o.tickets_per_grab) c.tickets_per_grab = grab_opts[ig];
                if (std::memcmp(&c, &cur, sizeof(c)) == 0) continue;
                double t = 0.0;
                st = timed(c, &t);
                if (st != BNS_OK) return st;
                if (t < cur_t * 0.98) {  // keep only clear gains
                    cur = c;
                    cur_t = t;
                }
            }
        }
    }
    st = try_depths();
    if (st != BNS_OK) return st;
    // Samples per work unit: a depth with too few tests to fill the device
    // cuts each test's samples into chunks counted by different groups; the
    // smallest chunk and the units aimed for per group set how far.
    if (!o.split_min_samples && !o.units_per_group) {
        const int32_t split_opts[] = {0, 2048, 8192, 16384, -1};
        const int32_t upg_opts[] = {0, 4, 16};
        const bns_options start2 = cur;
        for (int32_t sm : split_opts)
            for (int32_t up : upg_opts) {
                if (sm == -1 && up) continue;
                bns_options c = start2;
                c.split_min_samples = sm;
                c.units_per_group = up;
                if (std::memcmp(&c, &cur, sizeof(c)) == 0) continue;
                double t = 0.0;
                st = timed(c, &t);
                if (st != BNS_OK) return st;
                if (t < cur_t * 0.98) {
                    cur = c;
                    cur_t = t;
                }
            }
    }
    // Depth 1 in units of one test or of one edge's ranks of a level (the
    // latter with depth 1 in workgroup mode too, when the modes are tuned:
    // a wave's share of the LDS holds few of a unit's tables).
    if (o.group_tests == BNS_GROUP_AUTO) {
        std::vector<bns_options> cands;
        for (int32_t gt : {BNS_GROUP_TEST, BNS_GROUP_EDGE}) {
            bns_options c = cur;
            c.group_tests = gt;
            cands.push_back(c);
            if (gt == BNS_GROUP_EDGE && o.test_group == 0 && o.wave_depths == 0u && o.block_depths == 0u &&
                (cur.wave_depths & 2u)) {
                c.wave_depths &= ~2u;
                c.block_depths |= 2u;
                cands.push_back(c);
            }
        }
        for (const bns_options &c : cands) {
            if (std::memcmp(&c, &cur, sizeof(c)) == 0) continue;
            double t = 0.0;
            st = timed(c, &t);
            if (st != BNS_OK) return st;
            if (t < cur_t * 0.98) {
                cur = c;
                cur_t = t;
            }
        }
    }
    // Depth 1 in the test kernel or through the masked contractions.
    if (o.depth1 == BNS_DEPTH1_AUTO) {
        bns_options c = cur;
        c.depth1 = BNS_DEPTH1_GRAM;
        double t = 0.0;
        st = timed(c, &t);
        if (st != BNS_OK && st != BNS_E_NOMEM) return st;
        if (st == BNS_OK && t < cur_t * 0.98) {
            cur = c;
            cur_t = t;
        }
    }
    // Depth 0 in the test kernel or through the pair contraction.
    if (o.depth0 == BNS_DEPTH0_AUTO) {
        for (int32_t d0 : {BNS_DEPTH0_TESTS, BNS_DEPTH0_PAIRS}) {
            bns_options c = cur;
            c.depth0 = d0;
            double t = 0.0;
            st = timed(c, &t);
            if (st == BNS_E_NOMEM && d0 == BNS_DEPTH0_PAIRS) continue;  // tiles beyond the limit
            if (st != BNS_OK) return st;
            if (t < cur_t * 0.98) {
                cur = c;
                cur_t = t;
            }
        }
    }
    // The grab size again, and the groups per depth, under the paths chosen
    // last: edge units or contractions change the depth that dominated the
    // grid's searches.
    if (!o.tickets_per_grab) {
        const bns_options start3 = cur;
        for (int32_t g : grab_opts) {
            bns_options c = start3;
            c.tickets_per_grab = g;
            if (std::memcmp(&c, &cur, sizeof(c)) == 0) continue;
            double t = 0.0;
            st = timed(c, &t);
            if (st != BNS_OK) return st;
            if (t < cur_t * 0.98) {
                cur = c;
                cur_t = t;
            }
        }
        st = try_depths();
        if (st != BNS_OK) return st;
    }
    *best = cur;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.push_back(TuneEntry{device, key, cur});
    tune_save_entry(g_tune.back());
    return BNS_OK;
}

extern "C" bns_status bns_pc_skeleton_dataset(const bns_dataset *ds, double alpha, int32_t max_depth,
                                              const bns_options *opt, bns_skeleton **out) {
    if (!out) return fail(BNS_E_INVALID_ARG, "out is NULL");
    return bns_pc_skeleton_batch(&ds, 1, &alpha, &max_depth, opt, out);
}

extern "C" bns_status bns_pc_skeleton(const uint8_t *data, int64_t n_samples, int32_t n_vars,
                                      const uint8_t *cards, double alpha, int32_t max_depth,
                                      const bns_options *opt, bns_skeleton **out) {
    if (!out) return fail(BNS_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!(alpha > 0.0 && alpha < 1.0)) return fail(BNS_E_INVALID_ARG, "alpha must be in (0, 1)");
    if (max_depth < -1) return fail(BNS_E_INVALID_ARG, "max_depth must be >= -1");
    bns_options o;
    bns_status st = read_options(opt, &o);
    if (st != BNS_OK) return st;
    bns_dataset *ds = nullptr;
    st = bns_dataset_create(data, n_samples, n_vars, cards, &ds);
    if (st != BNS_OK) return st;
    st = bns_pc_skeleton_dataset(ds, alpha, max_depth, &o, out);
    bns_dataset_free(ds);
    return st;
}
