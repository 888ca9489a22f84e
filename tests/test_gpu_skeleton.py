"""GPU parity of the PC-stable skeleton (Algorithm 1) against the oracle.

Skeleton, removal depths and sepsets must be identical to the oracle's, and
the per-depth canonical test counts (tests in the sequential order up to each
edge's first accepting test) must equal the oracle's test counts, for the
batched form (FP32 + FP64 recheck, and FP64), the plain per-test form, with
and without graph replay, and across tile shapes.  The five synthetic
workloads are compared against stored oracle outputs (tests/golden/), smaller
random cases against the oracle run live.
"""

import numpy as np
import pytest

from bnsynth import make_config, make_dataset
from golden_util import compare_skeleton, compare_with_oracle, load_golden

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bns():
    import paper_2212_04259_amd as b
    b.load()
    return b


_CACHE = {}


def _cfg(k):
    if k not in _CACHE:
        _CACHE[k] = make_config(k)
    return _CACHE[k]


def _run(bns, ds, label, **opt):
    print(f"skeleton {label} n={ds.n_vars} m={ds.n_samples} opts={opt}", flush=True)
    o = bns.bns_options_default(**opt)
    return bns.bns_pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth, o)


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("prec", [0, 1])
def test_batched_matches_golden(bns, k, prec):
    g = load_golden(k)["datasets"][0]
    ds = _cfg(k)[0]
    assert ds.sha256() == g["sha256"]
    got = _run(bns, ds, f"cfg{k}", precision=prec)
    compare_skeleton(got, g, f"cfg{k} prec{prec}")


@pytest.mark.parametrize("k", [1, 2])
def test_plain_matches_golden(bns, k):
    g = load_golden(k)["datasets"][0]
    ds = _cfg(k)[0]
    got = _run(bns, ds, f"cfg{k} plain", form=bns.BNS_FORM_PLAIN, precision=1)
    compare_skeleton(got, g, f"cfg{k} plain")


@pytest.mark.parametrize("opts", [
    dict(lds_bytes=16384), dict(lds_bytes=32768, wg_per_cu=1), dict(lds_bytes=65536),
    dict(use_graph=0), dict(timing=1), dict(recheck_band=0.0),
    dict(split_min_samples=-1), dict(split_min_samples=1024, units_per_group=16),
    dict(split_min_samples=1024, units_per_group=16, lds_bytes=8192),
    dict(test_group=2), dict(test_group=2, split_min_samples=-1),
    dict(test_group=2, split_min_samples=1024, units_per_group=64),
    dict(test_group=1, split_min_samples=2048, units_per_group=4, precision=1),
    dict(max_replicas=1), dict(max_replicas=16, tickets_per_grab=8),
    dict(test_group=1, max_replicas=4, tickets_per_grab=1),
    dict(ticket_runs=1), dict(ticket_runs=2), dict(ticket_runs=2, test_group=1, tickets_per_grab=8),
    dict(ticket_runs=2, split_min_samples=1024, units_per_group=16),
])
def test_tile_shapes_and_modes_identical(bns, opts):
    g = load_golden(2)["datasets"][0]
    ds = _cfg(2)[0]
    got = _run(bns, ds, "cfg2", **opts)
    compare_skeleton(got, g, f"cfg2 {opts}")


@pytest.mark.parametrize("k", [1, 3])
def test_ticket_runs_match_golden(bns, k):
    # Tickets dealt to the grab counters in runs of 64 (the kernel instance
    # that large searches use) on small workloads.
    g = load_golden(k)["datasets"][0]
    got = _run(bns, _cfg(k)[0], f"cfg{k} runs", ticket_runs=2)
    compare_skeleton(got, g, f"cfg{k} ticket_runs=2")


@pytest.mark.parametrize("k", [1, 2])
def test_per_depth_groups_match_golden(bns, k):
    # Lanes per test chosen per depth (wave at even depths, workgroup at odd
    # ones, and the reverse) leave the skeleton and sepsets unchanged.
    g = load_golden(k)["datasets"][0]
    for wave, block in ((0x55555555, 0xAAAAAAAA), (0xAAAAAAAA, 0x55555555)):
        got = _run(bns, _cfg(k)[0], f"cfg{k} depths {wave:#x}", wave_depths=wave, block_depths=block)
        compare_skeleton(got, g, f"cfg{k} wave_depths={wave:#x}")


def test_large_search_results_copy_path(bns, orc):
    # 2,000 variables: the multi-workgroup preparation and removal kernels,
    # and results beyond what the last kernel publishes into host memory
    # (4 MB of removal depths, more removal records than the published
    # prefix), which are copied after the search.
    ds = make_dataset(2000, 2600, 3, 2, 3, 0.5, 400, seed=777, alpha=0.01)
    ref = orc.pc_skeleton(ds.data, ds.cards, ds.alpha, 1)
    for runs in (1, 2):
        print(f"skeleton n=2000 m=400 max_depth=1 ticket_runs={runs}", flush=True)
        o = bns.bns_options_default(ticket_runs=runs)
        got = bns.bns_pc_skeleton(ds.data, ds.cards, ds.alpha, 1, o)
        compare_with_oracle(got, ref, f"n=2000 ticket_runs={runs}")


def test_split_tables_stay_clean_across_searches(bns):
    # Merge tables of split depths are cleared by the group that evaluates
    # each test; back-to-back searches of different shapes must not see
    # leftovers.
    for k, opts in ((2, dict(split_min_samples=1024, units_per_group=32)),
                    (1, dict(split_min_samples=1024, units_per_group=32)),
                    (3, dict(split_min_samples=1024, units_per_group=8)),
                    (2, dict(split_min_samples=1024, units_per_group=32, test_group=2))):
        g = load_golden(k)["datasets"][0]
        got = _run(bns, _cfg(k)[0], f"cfg{k}", **opts)
        compare_skeleton(got, g, f"cfg{k} {opts}")


def test_cfg4_full_size(bns):
    g = load_golden(4)["datasets"][0]
    ds = _cfg(4)[0]
    assert ds.sha256() == g["sha256"]
    got = _run(bns, ds, "cfg4")
    compare_skeleton(got, g, "cfg4")


def test_cfg5_batch_of_64(bns):
    gold = load_golden(5)["datasets"]
    dss = _cfg(5)
    assert [d.sha256() for d in dss] == [g["sha256"] for g in gold]
    print(f"skeleton cfg5 batch of {len(dss)}", flush=True)
    handles = [bns.bns_dataset_create(d.data, d.cards) for d in dss]
    # default options, then chunks shorter than most datasets' sample counts
    # (ragged chunk counts per test within one depth)
    for opts in (dict(), dict(split_min_samples=3072, units_per_group=16), dict(ticket_runs=1)):
        print(f"  options {opts}", flush=True)
        o = bns.bns_options_default(**opts)
        outs = bns.bns_pc_skeleton_batch(handles, [d.alpha for d in dss],
                                         [d.max_depth for d in dss], o)
        assert len(outs) == len(dss)
        for i, (got, g) in enumerate(zip(outs, gold)):
            # each handle carries its own dataset's per-depth counters
            compare_skeleton(got, g, f"cfg5[{i}] {opts}")
            assert all(s["tests_executed"] >= s["tests_required"] for s in got.stats)
            assert all(s["edges"] >= s["removed"] for s in got.stats)


def test_small_batch_against_live_oracle(bns, orc):
    # A batch small enough for the one-workgroup preparation and removal
    # kernels (adjacency bit rows in LDS): per-problem counters come from
    # those kernels; sizes, alphas and depth limits differ per problem.
    dss, alphas, depths = [], [], []
    for k, (n, m, md, al) in enumerate([(7, 3000, -1, 0.05), (24, 20_000, -1, 0.01), (13, 1, -1, 0.05),
                                        (31, 9000, 1, 0.05), (2, 500, -1, 0.05), (40, 12_345, 2, 0.02)]):
        dss.append(make_dataset(n, int(1.3 * n), 3, 2, 4, 0.5, m, seed=9100 + k, alpha=al))
        alphas.append(al)
        depths.append(md)
    handles = [bns.bns_dataset_create(d.data, d.cards) for d in dss]
    print(f"skeleton small batch of {len(dss)}", flush=True)
    outs = bns.bns_pc_skeleton_batch(handles, alphas, depths)
    for k, (got, ds) in enumerate(zip(outs, dss)):
        ref = orc.pc_skeleton(ds.data, ds.cards, alphas[k], depths[k])
        compare_with_oracle(got, ref, f"small batch [{k}]")


@pytest.mark.parametrize("seed", range(6))
def test_random_small_against_live_oracle(bns, orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 16))
    m = int(rng.integers(1, 20_000))
    ds = make_dataset(n, int(1.3 * n), 3, 2, 5, 0.5, m, seed=4242 + seed, alpha=0.05)
    ref = orc.pc_skeleton(ds.data, ds.cards, ds.alpha, -1)
    for form in (0, 1):
        got = _run(bns, ds, f"random seed {seed}", form=form)
        compare_with_oracle(got, ref, f"random seed {seed} form {form}")


def test_max_depth_zero_and_one(bns, orc):
    ds = _cfg(2)[0]
    for md in (0, 1):
        ref = orc.pc_skeleton(ds.data, ds.cards, ds.alpha, md)
        print(f"skeleton cfg2 max_depth={md}", flush=True)
        got = bns.bns_pc_skeleton(ds.data, ds.cards, ds.alpha, md)
        compare_with_oracle(got, ref, f"cfg2 max_depth={md}")
        assert len(got.stats) == md + 1


def test_wrap_device_and_caller_stream(bns):
    import torch
    g = load_golden(2)["datasets"][0]
    ds = _cfg(2)[0]
    ld = (ds.n_samples + 63) // 64 * 64
    host = np.zeros((ds.n_vars, ld), dtype=np.uint8)
    host[:, :ds.n_samples] = ds.data
    dev = torch.from_numpy(host).to("cuda:0")
    print("skeleton cfg2 wrapped device tensor", flush=True)
    h = bns.bns_dataset_wrap_device(dev, ds.n_samples, ds.cards)
    s = torch.cuda.Stream()
    o = bns.bns_options_default(stream=s.cuda_stream)
    got = bns.bns_pc_skeleton_dataset(h, ds.alpha, ds.max_depth, o)
    compare_skeleton(got, g, "cfg2 wrapped")
    bad = dev.clone()
    bad[5, 17] = 200
    with pytest.raises(bns.BnsError) as ei:
        bns.bns_dataset_wrap_device(bad, ds.n_samples, ds.cards)
    assert "sample 17" in str(ei.value)


def test_autotune_options_keep_results(bns):
    # The autotuner only chooses launch options: searches with its choice
    # match the oracle, and a second call for the same workload is cached.
    import time
    g = load_golden(1)["datasets"][0]
    ds = _cfg(1)[0]
    h = bns.bns_dataset_create(ds.data, ds.cards)
    print("autotune cfg1", flush=True)
    best = bns.bns_autotune([h], [ds.alpha], [ds.max_depth], trials=1)
    assert best.test_group in (0, 1, 2) and best.max_replicas in (0, 16, 64)
    t0 = time.perf_counter()
    again = bns.bns_autotune([h], [ds.alpha], [ds.max_depth], trials=1)
    assert time.perf_counter() - t0 < 0.05
    assert (again.test_group, again.max_replicas, again.lds_bytes, again.tickets_per_grab) == \
        (best.test_group, best.max_replicas, best.lds_bytes, best.tickets_per_grab)
    got = bns.bns_pc_skeleton_dataset(h, ds.alpha, ds.max_depth, best)
    compare_skeleton(got, g, "cfg1 autotuned")
