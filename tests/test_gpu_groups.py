"""GPU parity of depth 1 in (edge, level) units (options.group_tests =
BNS_GROUP_EDGE: the ranks an edge has in one level of the work queue are
counted in one pass that loads X and Y once, the counterpart of Section
IV-B's group of tests of one edge) against the oracle.

The level structure and the first-accept rule are unchanged, so skeleton,
removal depths, sepsets and per-depth canonical counts must equal the
oracle's: on the five workloads (stored results) and on random datasets run
live — ragged sample counts (the per-sample tail of the packed count), edges
with many ranks per level (several passes of up to eight tests, stopping
after an acceptance), cardinalities up to 8 (fewer tables per pass), one
wave or one workgroup per unit, replication caps, FP64, the other
statistics, graph replay off and event timing.
"""

import numpy as np
import pytest

from bnsynth import make_config, make_dataset
from golden_util import compare_skeleton, compare_with_oracle, load_golden

pytestmark = pytest.mark.gpu

EDGE = 2


@pytest.fixture(scope="module")
def bns():
    import paper_2212_04259_amd as b
    b.load()
    return b


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_edge_units_match_golden(bns, k):
    g = load_golden(k)["datasets"][0]
    ds = make_config(k)[0]
    print(f"edge units cfg{k}", flush=True)
    got = bns.bns_pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth, bns.bns_options_default(group_tests=EDGE))
    compare_skeleton(got, g, f"cfg{k} group_tests=edge")


def test_edge_units_batch_of_64(bns):
    gold = load_golden(5)["datasets"]
    dss = make_config(5)
    print("edge units cfg5 batch of 64", flush=True)
    hs = [bns.bns_dataset_create(d.data, d.cards) for d in dss]
    outs = bns.bns_pc_skeleton_batch(hs, [d.alpha for d in dss], [d.max_depth for d in dss],
                                     bns.bns_options_default(group_tests=EDGE))
    for i, (got, g) in enumerate(zip(outs, gold)):
        compare_skeleton(got, g, f"cfg5[{i}] group_tests=edge")


@pytest.mark.parametrize("m", [1, 15, 17, 255, 4097, 12_295])
def test_edge_units_ragged_samples(bns, orc, m):
    ds = make_dataset(23, 45, 3, 2, 5, 0.5, m, seed=8000 + m)
    ref = orc.pc_skeleton(ds.data, ds.cards, 0.05, -1)
    print(f"edge units ragged m={m}", flush=True)
    got = bns.bns_pc_skeleton(ds.data, ds.cards, 0.05, -1, bns.bns_options_default(group_tests=EDGE))
    compare_with_oracle(got, ref, f"edge units m={m}")


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("test_group", [1, 2])
def test_edge_units_many_ranks_wide_cards(bns, orc, seed, test_group):
    # a dense DAG with cardinalities up to 8: edges keep many neighbours after
    # depth 0 (levels of 8, 16, 32 ranks: several passes per unit) and tables
    # up to 512 cells (fewer tests per pass, less replication)
    ds = make_dataset(36, 200, 10, 2, 8, 0.3, 20_000, seed=8100 + seed)
    ref = orc.pc_skeleton(ds.data, ds.cards, 0.05, 2)
    print(f"edge units dense seed={seed} test_group={test_group}", flush=True)
    o = bns.bns_options_default(group_tests=EDGE, test_group=test_group)
    got = bns.bns_pc_skeleton(ds.data, ds.cards, 0.05, 2, o)
    compare_with_oracle(got, ref, f"edge units dense seed={seed} test_group={test_group}")


@pytest.mark.parametrize("extra", [dict(precision=1), dict(use_graph=0), dict(timing=1), dict(max_replicas=1),
                                   dict(max_replicas=64), dict(lds_bytes=8192)])
def test_edge_units_options(bns, orc, extra):
    ds = make_dataset(30, 50, 3, 2, 5, 0.5, 30_000, seed=8200)
    ref = orc.pc_skeleton(ds.data, ds.cards, 0.05, -1)
    print(f"edge units {extra}", flush=True)
    got = bns.bns_pc_skeleton(ds.data, ds.cards, 0.05, -1, bns.bns_options_default(group_tests=EDGE, **extra))
    compare_with_oracle(got, ref, f"edge units {extra}")


@pytest.mark.parametrize("stat,df_rule", [(1, 0), (0, 1), (1, 1)])
def test_edge_units_other_statistics(bns, orc, stat, df_rule):
    ds = make_config(2)[0]
    ref = orc.pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth, statistic=stat, df_rule=df_rule)
    print(f"edge units cfg2 stat={stat} df_rule={df_rule}", flush=True)
    o = bns.bns_options_default(group_tests=EDGE, statistic=stat, df_rule=df_rule)
    got = bns.bns_pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth, o)
    compare_with_oracle(got, ref, f"edge units stat={stat} df_rule={df_rule}")
    sparse = make_dataset(12, 20, 3, 3, 6, 0.5, 90, seed=8300)
    ref = orc.pc_skeleton(sparse.data, sparse.cards, 0.05, -1, statistic=stat, df_rule=df_rule)
    got = bns.bns_pc_skeleton(sparse.data, sparse.cards, 0.05, -1, o)
    compare_with_oracle(got, ref, f"edge units sparse stat={stat} df_rule={df_rule}")


def test_edge_units_tickets_count_edges_per_level(bns):
    # in (edge, level) units a level holds one unit per edge that has ranks
    # in it: depth 1's work units are fewer than its tests
    ds = make_config(2)[0]
    got = bns.bns_pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth, bns.bns_options_default(group_tests=EDGE))
    base = bns.bns_pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth, bns.bns_options_default())
    assert got.stats[1]["tickets"] < base.stats[1]["tickets"]
    assert got.stats[1]["tests_required"] == base.stats[1]["tests_required"]
    for d in (0, 2):
        assert got.stats[d]["tickets"] == base.stats[d]["tickets"]

