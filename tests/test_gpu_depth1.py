"""GPU parity of depth 1 through the masked Gram contractions (options.depth1 =
BNS_DEPTH1_GRAM: every depth-1 table as a block of G_c = H^T diag(X_u = c) H
over the one-hot columns H of a node's frozen neighbours, on int8 MFMA)
against the oracle.

Every depth-1 test is evaluated and each edge keeps its first accepting
test, so skeleton, removal depths, sepsets and per-depth canonical counts
must equal the oracle's: on the five workloads (stored results), together
with the depth-0 contraction, and on random datasets run live — ragged sample
counts (sample chunks and their edges), nodes whose neighbours take several
tile blocks, the other statistics, FP64, graph replay off and event timing.
Cardinalities above 8 and verification mode keep the test kernel.
"""

import numpy as np
import pytest

from bnsynth import make_config, make_dataset
from golden_util import compare_skeleton, compare_with_oracle, load_golden

pytestmark = pytest.mark.gpu

GRAM = 2


@pytest.fixture(scope="module")
def bns():
    import paper_2212_04259_amd as b
    b.load()
    return b


def _depth1_tests(got):
    """Every test of depth 1: each node u owns deg(u) (deg(u) - 1) of them
    (an edge (u, y) conditioned on each other neighbour), deg over the pairs
    that depth 0 kept."""
    n = got.adj.shape[0]
    alive1 = (np.asarray(got.depth) != 0) & ~np.eye(n, dtype=bool)
    deg = alive1.sum(1).astype(np.int64)
    return int((deg * (deg - 1)).sum())


def _depth1_ran_gram(got):
    s1 = got.stats[1]
    assert s1["test_group"] == 3, s1  # the contraction ran depth 1
    assert s1["tests_executed"] == _depth1_tests(got), s1  # every test of the depth was evaluated


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_depth1_gram_matches_golden(bns, k):
    g = load_golden(k)["datasets"][0]
    ds = make_config(k)[0]
    print(f"depth1 gram cfg{k}", flush=True)
    got = bns.bns_pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth, bns.bns_options_default(depth1=GRAM))
    compare_skeleton(got, g, f"cfg{k} depth1=gram")
    _depth1_ran_gram(got)


@pytest.mark.parametrize("k", [3, 4])
def test_both_contractions_match_golden(bns, k):
    g = load_golden(k)["datasets"][0]
    ds = make_config(k)[0]
    print(f"depth0 pairs + depth1 gram cfg{k}", flush=True)
    got = bns.bns_pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth,
                              bns.bns_options_default(depth0=2, depth1=GRAM))
    compare_skeleton(got, g, f"cfg{k} both contractions")
    assert got.stats[0]["test_group"] == 3
    _depth1_ran_gram(got)


def test_depth1_gram_batch_of_64(bns):
    gold = load_golden(5)["datasets"]
    dss = make_config(5)
    print("depth1 gram cfg5 batch of 64", flush=True)
    hs = [bns.bns_dataset_create(d.data, d.cards) for d in dss]
    outs = bns.bns_pc_skeleton_batch(hs, [d.alpha for d in dss], [d.max_depth for d in dss],
                                     bns.bns_options_default(depth1=GRAM))
    for i, (got, g) in enumerate(zip(outs, gold)):
        compare_skeleton(got, g, f"cfg5[{i}] depth1=gram")
        if len(got.stats) > 1 and got.stats[1]["tests_executed"] > 0:
            _depth1_ran_gram(got)


@pytest.mark.parametrize("m", [1, 63, 65, 4095, 4097, 12_345, 40_003])
def test_depth1_gram_ragged_samples(bns, orc, m):
    ds = make_dataset(23, 45, 3, 2, 5, 0.5, m, seed=7000 + m)
    print(f"depth1 gram ragged m={m}", flush=True)
    for md in (1, -1):
        ref = orc.pc_skeleton(ds.data, ds.cards, 0.05, md)
        got = bns.bns_pc_skeleton(ds.data, ds.cards, 0.05, md, bns.bns_options_default(depth1=GRAM))
        compare_with_oracle(got, ref, f"depth1 gram m={m} max_depth={md}")


@pytest.mark.parametrize("seed", range(3))
def test_depth1_gram_several_tile_blocks(bns, orc, seed):
    # a dense DAG: after depth 0 nodes keep many neighbours, whose one-hot
    # rows span several 64-row tile blocks
    ds = make_dataset(40, 260, 12, 3, 6, 0.3, 20_000, seed=7100 + seed)
    ref = orc.pc_skeleton(ds.data, ds.cards, 0.05, 1)
    # one-hot rows of each node's neighbours at depth 1 (pairs not removed at
    # depth 0): some node needs more than one 64-row block
    alive1 = (ref.depth != 0) & ~np.eye(ds.n_vars, dtype=bool)
    rows = alive1.astype(np.int64) @ ds.cards.astype(np.int64)
    assert rows.max() > 64, rows.max()
    print(f"depth1 gram dense seed={seed} max rows {rows.max()}", flush=True)
    got = bns.bns_pc_skeleton(ds.data, ds.cards, 0.05, 1, bns.bns_options_default(depth1=GRAM))
    compare_with_oracle(got, ref, f"depth1 gram dense seed={seed}")
    _depth1_ran_gram(got)


@pytest.mark.parametrize("extra", [dict(precision=1), dict(use_graph=0), dict(timing=1)])
def test_depth1_gram_options(bns, orc, extra):
    ds = make_dataset(30, 50, 3, 2, 5, 0.5, 30_000, seed=7200)
    ref = orc.pc_skeleton(ds.data, ds.cards, 0.05, -1)
    print(f"depth1 gram {extra}", flush=True)
    got = bns.bns_pc_skeleton(ds.data, ds.cards, 0.05, -1, bns.bns_options_default(depth1=GRAM, **extra))
    compare_with_oracle(got, ref, f"depth1 gram {extra}")
    _depth1_ran_gram(got)
    if extra.get("timing"):
        assert got.stats[1]["kernel_seconds"] > 0.0


@pytest.mark.parametrize("stat,df_rule", [(1, 0), (0, 1), (1, 1)])
def test_depth1_gram_other_statistics(bns, orc, stat, df_rule):
    ds = make_config(2)[0]
    ref = orc.pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth, statistic=stat, df_rule=df_rule)
    print(f"depth1 gram cfg2 stat={stat} df_rule={df_rule}", flush=True)
    o = bns.bns_options_default(depth1=GRAM, statistic=stat, df_rule=df_rule)
    got = bns.bns_pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth, o)
    compare_with_oracle(got, ref, f"depth1 gram stat={stat} df_rule={df_rule}")
    # few samples over many cells: empty categories and strata
    sparse = make_dataset(12, 20, 3, 3, 6, 0.5, 90, seed=7300)
    ref = orc.pc_skeleton(sparse.data, sparse.cards, 0.05, -1, statistic=stat, df_rule=df_rule)
    got = bns.bns_pc_skeleton(sparse.data, sparse.cards, 0.05, -1, o)
    compare_with_oracle(got, ref, f"depth1 gram sparse stat={stat} df_rule={df_rule}")


def test_depth1_wide_cardinalities_keep_the_test_kernel(bns, orc):
    ds = make_dataset(20, 30, 2, 2, 12, 0.7, 10_000, seed=7400)
    assert ds.cards.max() > 8
    ref = orc.pc_skeleton(ds.data, ds.cards, 0.05, 1)
    got = bns.bns_pc_skeleton(ds.data, ds.cards, 0.05, 1, bns.bns_options_default(depth1=GRAM))
    compare_with_oracle(got, ref, "depth1 wide cards")
    assert got.stats[1]["test_group"] in (1, 2)


def test_depth1_with_report_errors_keeps_the_test_kernel(bns):
    ds = make_config(1)[0]
    got = bns.bns_pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth,
                              bns.bns_options_default(depth1=GRAM, report_errors=1))
    assert got.stats[1]["test_group"] in (1, 2)
    assert got.stats[1]["err_tests"] == got.stats[1]["tests_executed"]
