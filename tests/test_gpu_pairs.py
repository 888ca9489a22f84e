"""GPU parity of depth 0 through the pair contraction (options.depth0 =
BNS_DEPTH0_PAIRS: every pairwise table as a block of the one-hot Gram matrix
on int8 MFMA, Section IV-B's depth 0 of one test per pair) against the oracle.

Skeleton, removal depths, sepsets and per-depth counts identical to the
oracle's on the five workloads (stored results) and on random datasets run
live: cardinalities above 8 (the byte-compare expansion), ragged sample
counts around the 64-sample steps and the chunk boundaries, device data with
valid-looking bytes past the last sample, graph replay off and event timing,
and the other statistics.
"""

import numpy as np
import pytest

from bnsynth import make_config, make_dataset
from golden_util import compare_skeleton, compare_with_oracle, load_golden

pytestmark = pytest.mark.gpu

PAIRS = 2


@pytest.fixture(scope="module")
def bns():
    import paper_2212_04259_amd as b
    b.load()
    return b


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_pairs_match_golden(bns, k):
    g = load_golden(k)["datasets"][0]
    ds = make_config(k)[0]
    print(f"pairs cfg{k}", flush=True)
    o = bns.bns_options_default(depth0=PAIRS)
    got = bns.bns_pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth, o)
    compare_skeleton(got, g, f"cfg{k} depth0=pairs")
    s0 = got.stats[0]
    assert s0["tests_executed"] == s0["tests_required"] == s0["edges"] == ds.n_vars * (ds.n_vars - 1) // 2


def test_pairs_batch_of_64(bns):
    gold = load_golden(5)["datasets"]
    dss = make_config(5)
    print("pairs cfg5 batch of 64", flush=True)
    hs = [bns.bns_dataset_create(d.data, d.cards) for d in dss]
    outs = bns.bns_pc_skeleton_batch(hs, [d.alpha for d in dss], [d.max_depth for d in dss],
                                     bns.bns_options_default(depth0=PAIRS))
    for i, (got, g) in enumerate(zip(outs, gold)):
        compare_skeleton(got, g, f"cfg5[{i}] depth0=pairs")


@pytest.mark.parametrize("m", [1, 15, 63, 64, 65, 127, 2047, 2049, 8191, 40_003])
def test_pairs_ragged_samples(bns, orc, m):
    ds = make_dataset(23, 30, 3, 2, 5, 0.5, m, seed=6000 + m)
    ref = orc.pc_skeleton(ds.data, ds.cards, 0.05, 1)
    print(f"pairs ragged m={m}", flush=True)
    got = bns.bns_pc_skeleton(ds.data, ds.cards, 0.05, 1, bns.bns_options_default(depth0=PAIRS))
    compare_with_oracle(got, ref, f"pairs m={m}")


@pytest.mark.parametrize("seed", range(3))
def test_pairs_wide_cardinalities(bns, orc, seed):
    # cardinalities up to 20: variables above 8 categories take the
    # byte-compare expansion; mixed with narrow ones in one tile
    ds = make_dataset(30, 40, 2, 2, 20, 0.7, 30_000, seed=6100 + seed)
    assert ds.cards.max() > 8 and ds.cards.min() <= 8
    ref = orc.pc_skeleton(ds.data, ds.cards, 0.05, 1)
    print(f"pairs wide cards seed={seed}", flush=True)
    for extra in (dict(), dict(precision=1), dict(use_graph=0), dict(timing=1)):
        got = bns.bns_pc_skeleton(ds.data, ds.cards, 0.05, 1, bns.bns_options_default(depth0=PAIRS, **extra))
        compare_with_oracle(got, ref, f"pairs wide seed={seed} {extra}")


def test_pairs_wrapped_device_data_with_padding_bytes(bns, orc):
    import torch
    ds = make_dataset(17, 20, 3, 2, 4, 0.5, 3_001, seed=6200)
    ld = (ds.n_samples + 15) // 16 * 16 + 48
    host = np.full((ds.n_vars, ld), 1, dtype=np.uint8)  # a valid category past the last sample
    host[:, :ds.n_samples] = ds.data
    dev = torch.from_numpy(host).to("cuda:0")
    h = bns.bns_dataset_wrap_device(dev, ds.n_samples, ds.cards)
    ref = orc.pc_skeleton(ds.data, ds.cards, 0.05, -1)
    print("pairs wrapped device data", flush=True)
    got = bns.bns_pc_skeleton_dataset(h, 0.05, -1, bns.bns_options_default(depth0=PAIRS))
    compare_with_oracle(got, ref, "pairs wrapped")


@pytest.mark.parametrize("stat,df_rule", [(1, 0), (0, 1), (1, 1)])
def test_pairs_other_statistics(bns, orc, stat, df_rule):
    ds = make_config(2)[0]
    ref = orc.pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth, statistic=stat, df_rule=df_rule)
    print(f"pairs cfg2 stat={stat} df_rule={df_rule}", flush=True)
    o = bns.bns_options_default(depth0=PAIRS, statistic=stat, df_rule=df_rule)
    got = bns.bns_pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth, o)
    compare_with_oracle(got, ref, f"pairs stat={stat} df_rule={df_rule}")
    sparse = make_dataset(12, 16, 3, 3, 6, 0.5, 90, seed=6300)
    ref = orc.pc_skeleton(sparse.data, sparse.cards, 0.05, -1, statistic=stat, df_rule=df_rule)
    got = bns.bns_pc_skeleton(sparse.data, sparse.cards, 0.05, -1, o)
    compare_with_oracle(got, ref, f"pairs sparse stat={stat} df_rule={df_rule}")


def test_pairs_with_report_errors_keeps_the_test_kernel(bns):
    # verification mode compares the FP32 statistic with FP64 on every test,
    # so depth 0 stays in the test kernel
    ds = make_config(1)[0]
    got = bns.bns_pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth,
                              bns.bns_options_default(depth0=PAIRS, report_errors=1))
    assert got.stats[0]["err_tests"] == got.stats[0]["tests_executed"]


def _check_pairs(bns, orc, ds, alpha, stat=0, df_rule=0, sample=None, seed=0):
    h = bns.bns_dataset_create(ds.data, ds.cards)
    o = bns.bns_options_default(statistic=stat, df_rule=df_rule)
    r = bns.bns_ci_pairs(h, alpha, o)
    n = ds.n_vars
    assert len(r["stat"]) == n * (n - 1) // 2
    idx = range(len(r["pairs"]))
    if sample is not None and sample < len(r["pairs"]):
        idx = np.random.default_rng(seed).choice(len(r["pairs"]), size=sample, replace=False)
    for q in idx:
        i, j = r["pairs"][q]
        s, df, p = orc.ci_test(ds.data, ds.cards, i, j, (), statistic=stat, df_rule=df_rule)
        assert r["df"][q] == df, (i, j)
        assert abs(r["stat"][q] - s) <= 1e-9 * max(abs(s), 1.0), (i, j, r["stat"][q], s)
        assert abs(r["p"][q] - p) <= 1e-9 * max(p, 1e-300) + 1e-15, (i, j, r["p"][q], p)
        if abs(p - alpha) > 1e-9:
            assert bool(r["flags"][q] & 1) == (p > alpha), (i, j)
    return r


@pytest.mark.parametrize("m", [1, 63, 65, 4097, 50_000])
def test_ci_pairs_match_oracle(bns, orc, m):
    ds = make_dataset(25, 30, 3, 2, 5, 0.5, m, seed=6400 + m)
    print(f"ci_pairs m={m}", flush=True)
    _check_pairs(bns, orc, ds, 0.05)


@pytest.mark.parametrize("stat,df_rule", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_ci_pairs_wide_cards_large_df(bns, orc, stat, df_rule):
    # cardinalities up to 20: df up to 361 (the series and continued-fraction
    # tails) and the byte-compare expansion
    ds = make_dataset(20, 26, 2, 2, 20, 0.6, 20_000, seed=6500)
    print(f"ci_pairs wide stat={stat} df_rule={df_rule}", flush=True)
    r = _check_pairs(bns, orc, ds, 0.05, stat, df_rule)
    assert r["df"].max() > 128


def test_ci_pairs_sparse_adjusted(bns, orc):
    ds = make_dataset(16, 20, 3, 3, 7, 0.5, 60, seed=6600)
    for stat in (0, 1):
        _check_pairs(bns, orc, ds, 0.05, stat, 1)


def test_ci_pairs_full_size_samples(bns, orc):
    # the 1,000-variable, 200,000-sample workload: all 499,500 pairs in one
    # call, checked on a seeded sample of pairs
    ds = make_config(4)[0]
    print("ci_pairs cfg4 (sampled)", flush=True)
    _check_pairs(bns, orc, ds, ds.alpha, sample=300, seed=1)
