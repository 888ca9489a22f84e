"""Pins of the oracle's PC-stable driver (Algorithm 1, Sections IV-B and IV-C).

- Test order: the conditioning sets an edge is tested on, and their order, are
  compared with ``itertools.combinations`` over the frozen adjacency sets
  (lower-id endpoint's side first, lexicographic, one marginal test per pair
  at depth 0, side-B duplicates not removed).
- Logic: with a d-separation CI source on random DAGs, PC-stable must return
  the DAG's skeleton exactly and every sepset must d-separate (the textbook
  consistency of PC with a perfect independence oracle).
- Statistics: exact skeleton recovery from faithful small DAGs at large m, and
  invariance of skeleton and removal depths under relabelling the variables.
"""

import itertools

import networkx as nx
import numpy as np
import pytest

from bnsynth import forward_sample, make_dataset


def _dsep_source(dag):
    def p(x, y, s):
        return 1.0 if nx.is_d_separator(dag, {x}, {y}, set(s)) else 0.0
    return p


def _random_dag(rng, n, max_indeg, p_edge=0.35):
    order = rng.permutation(n)
    g = nx.DiGraph()
    g.add_nodes_from(range(n))
    for b in range(n):
        cands = [int(order[a]) for a in range(b)]
        rng.shuffle(cands)
        k = 0
        for c in cands:
            if k < max_indeg and rng.random() < p_edge:
                g.add_edge(c, int(order[b]))
                k += 1
    return g


@pytest.mark.parametrize("seed", range(25))
def test_dsep_oracle_recovers_skeleton(orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 13))
    dag = _random_dag(rng, n, 3)
    res = orc.pc_skeleton_cb(n, _dsep_source(dag), alpha=0.5)
    truth = np.zeros((n, n), dtype=np.uint8)
    for a, b in dag.edges():
        truth[a, b] = truth[b, a] = 1
    assert np.array_equal(res.adj, truth)
    for (i, j), S in res.sepsets.items():
        assert not truth[i, j]
        assert nx.is_d_separator(dag, {i}, {j}, set(S))
        assert len(S) == res.depth[i, j]
        assert list(S) == sorted(S)


def test_depth0_single_test_per_pair_and_stop(orc):
    calls = []

    def p(x, y, s):
        calls.append((x, y, s))
        return 0.0
    n = 5
    # Every test rejects independence: the graph stays complete, so depth d
    # runs C(3, d) tests per side for every pair while d <= n - 2.
    res = orc.pc_skeleton_cb(n, p, alpha=0.05)
    npairs = n * (n - 1) // 2
    d0 = [c for c in calls if len(c[2]) == 0]
    assert len(d0) == npairs
    assert d0 == [(i, j, ()) for i in range(n) for j in range(i + 1, n)]
    for d in range(1, n - 1):
        want = npairs * 2 * len(list(itertools.combinations(range(n - 2), d)))
        assert res.tests[d] == want
    assert res.n_depths == n - 1  # depth n-1 would need |a(v)\{u}| >= n-1: stop


@pytest.mark.parametrize("seed", range(6))
def test_test_order_is_grouped_lexicographic(orc, seed):
    """Record every query; rebuild the expected sequence from the frozen
    adjacency sets with itertools."""
    rng = np.random.default_rng(50 + seed)
    n = 7
    indep = {}
    calls = []

    def p(x, y, s):
        calls.append((x, y, s))
        key = (x, y, s)
        if key not in indep:
            indep[key] = rng.random() < 0.25
        return 1.0 if indep[key] else 0.0
    res = orc.pc_skeleton_cb(n, p, alpha=0.5)

    # Replay with the recorded answers to produce the expected call sequence.
    adj = np.ones((n, n), dtype=bool)
    np.fill_diagonal(adj, False)
    expected = []
    d = 0
    while True:
        snap = {v: [u for u in range(n) if adj[v, u]] for v in range(n)}
        if not any(adj[i, j] and (d == 0 or len(snap[i]) - 1 >= d or len(snap[j]) - 1 >= d)
                   for i in range(n) for j in range(i + 1, n)):
            break
        for i in range(n):
            for j in range(i + 1, n):
                if not adj[i, j]:
                    continue
                if d == 0:
                    cands = [()]
                else:
                    A = [u for u in snap[i] if u != j]
                    B = [u for u in snap[j] if u != i]
                    cands = list(itertools.combinations(A, d)) + list(itertools.combinations(B, d))
                for S in cands:
                    expected.append((i, j, S))
                    if indep[(i, j, S)]:
                        adj[i, j] = adj[j, i] = False
                        assert res.sepsets[(i, j)] == S
                        assert res.depth[i, j] == d
                        break
        d += 1
    assert calls == expected
    assert sum(res.tests) == len(expected)


def test_max_depth_limits_depths(orc):
    n = 6
    res = orc.pc_skeleton_cb(n, lambda x, y, s: 0.0, alpha=0.05, max_depth=2)
    assert res.n_depths == 3


def test_tie_p_equal_alpha_is_dependent(orc):
    res = orc.pc_skeleton_cb(4, lambda x, y, s: 0.05, alpha=0.05, max_depth=0)
    assert res.adj.sum() == 4 * 3


def _strong_cpts(rng, cards, parents, gap=0.6):
    """CPT rows concentrated on a category that grows monotonically with the
    sum of the parent values, so every parent is marginally dependent on the
    child (a faithful, strong network)."""
    cpts = []
    for v, r in enumerate(cards):
        pc = [int(cards[p]) for p in parents[v]]
        n_cfg = int(np.prod(pc)) if pc else 1
        top = max(1, sum(c - 1 for c in pc))
        rows = np.full((n_cfg, int(r)), (1 - gap) / int(r))
        for c in range(n_cfg):
            vals, rest = [], c
            for card in pc:                      # first parent fastest
                vals.append(rest % card)
                rest //= card
            cat = min(int(r) - 1, int(sum(vals) / top * int(r)))
            rows[c, cat] += gap
        cpts.append(rows)
    return cpts


@pytest.mark.parametrize("name,edges,n", [
    ("chain", [(0, 1), (1, 2), (2, 3)], 4),
    ("fork", [(1, 0), (1, 2)], 3),
    ("collider", [(0, 2), (1, 2)], 3),
    ("diamond", [(0, 1), (0, 2), (1, 3), (2, 3)], 4),
])
def test_exact_recovery_small_faithful_dags(orc, name, edges, n):
    rng = np.random.default_rng(7)
    cards = np.array([2, 3, 2, 3][:n], dtype=np.uint8)
    parents = [sorted(p for p, c in edges if c == v) for v in range(n)]
    order = list(nx.topological_sort(nx.DiGraph(edges)))
    order += [v for v in range(n) if v not in order]
    cpts = _strong_cpts(rng, cards, parents)
    data = forward_sample(rng, order, parents, cards, cpts, 200_000)
    res = orc.pc_skeleton(data, cards, alpha=0.01)
    truth = np.zeros((n, n), dtype=np.uint8)
    for a, b in edges:
        truth[a, b] = truth[b, a] = 1
    assert np.array_equal(res.adj, truth), name
    if name == "collider":
        assert res.sepsets[(0, 1)] == ()
    if name == "chain":
        assert res.sepsets[(0, 2)] == (1,)
        assert res.sepsets[(1, 3)] == (2,)


def test_exact_recovery_random_8var(orc):
    rng = np.random.default_rng(11)
    n = 8
    edges = [(0, 3), (1, 3), (3, 5), (2, 4), (4, 6), (5, 7), (6, 7)]
    cards = rng.integers(2, 4, n).astype(np.uint8)
    parents = [sorted(p for p, c in edges if c == v) for v in range(n)]
    order = list(nx.topological_sort(nx.DiGraph(edges)))
    cpts = _strong_cpts(rng, cards, parents)
    data = forward_sample(rng, order, parents, cards, cpts, 300_000)
    res = orc.pc_skeleton(data, cards, alpha=0.01)
    truth = np.zeros((n, n), dtype=np.uint8)
    for a, b in edges:
        truth[a, b] = truth[b, a] = 1
    assert np.array_equal(res.adj, truth)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_order_independence_under_relabelling(orc, seed):
    ds = make_dataset(14, 18, 3, 2, 4, 0.5, 8000, seed=9000 + seed)
    res = orc.pc_skeleton(ds.data, ds.cards, alpha=0.05)
    perm = np.random.default_rng(seed).permutation(ds.n_vars)   # new id -> old id
    inv = np.argsort(perm)                                      # old id -> new id
    res2 = orc.pc_skeleton(ds.data[perm], ds.cards[perm], alpha=0.05)
    assert res.knife_edges == 0 and res2.knife_edges == 0
    n = ds.n_vars
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            a, b = inv[i], inv[j]
            assert res.adj[i, j] == res2.adj[a, b]
            assert res.depth[i, j] == res2.depth[a, b]
    # Each relabelled sepset is a valid accepting set of the same size.
    for (a, b), S in res2.sepsets.items():
        i, j = int(perm[a]), int(perm[b])
        S_old = [int(perm[s]) for s in S]
        assert len(S_old) == res.depth[min(i, j), max(i, j)]
        p = orc.ci_test(ds.data, ds.cards, i, j, S_old)[2]
        assert p > 0.05


# ---------------------------------------------------------------------------
# Reading R16: the driver reports the closest p-value to alpha over every test
# it ran (min |p - alpha|) and the number of knife-edge tests (|p - alpha| <
# 1e-9).  A p-value source with planted gaps fixes both figures: which tests
# run is fixed by Algorithm 1 (one marginal test per pair at depth 0, then the
# frozen-set subsets), and only the planted tests come near alpha.
# ---------------------------------------------------------------------------
def _planted_source(plan, default=0.0):
    calls = []

    def p(x, y, s):
        calls.append((x, y, s))
        return plan.get((x, y, s), default)
    return p, calls


def test_knife_edge_report_planted_gaps(orc):
    a = 0.05
    plan = {
        (0, 1, ()): a + 4e-10,   # independent, knife edge
        (0, 2, ()): a - 2e-10,   # dependent, knife edge, the closest
        (0, 3, ()): a + 2e-9,    # independent, not a knife edge (gap 2e-9)
        (2, 3, ()): a - 3e-9,    # dependent, not a knife edge
    }
    src, calls = _planted_source(plan)
    res = orc.pc_skeleton_cb(4, src, alpha=a)
    # every planted test ran, at depth 0
    for key in plan:
        assert key in calls
    assert res.knife_edges == 2
    assert res.min_gap == abs((a - 2e-10) - a)
    # the decisions the planted values imply (strict p > alpha)
    assert not res.adj[0, 1] and not res.adj[0, 3]
    assert res.adj[0, 2] and res.adj[2, 3]


def test_knife_edge_report_counts_ties_and_later_depths(orc):
    a = 0.05
    # depth 0 removes nothing; at depth 1 the tie p == alpha is a knife edge
    # with gap 0 (and dependent, R4).  S = {0} is also the first subset of
    # side B of edge 1-2 (a(2) minus 1 = {0, 3}), and side-B repeats are run
    # (R11): the tie is met twice.  One more planted gap sits at 5e-10.
    plan = {(1, 2, (0,)): a, (0, 3, (1,)): a + 5e-10}
    src, calls = _planted_source(plan)
    res = orc.pc_skeleton_cb(4, src, alpha=a, max_depth=1)
    assert calls.count((1, 2, (0,))) == 2 and (0, 3, (1,)) in calls
    assert res.knife_edges == 3
    assert res.min_gap == 0.0
    assert res.adj[1, 2]            # the tie does not remove the edge
    assert not res.adj[0, 3]        # p slightly above alpha does
    assert res.depth[0, 3] == 1 and res.sepsets[(0, 3)] == (1,)


def test_knife_edge_report_far_from_alpha(orc):
    # no test near alpha: no knife edge, and the gap is the smallest planted one
    a = 0.01
    plan = {(0, 1, ()): 0.5, (1, 2, ()): a + 0.0025}
    src, _ = _planted_source(plan, default=1e-6)
    res = orc.pc_skeleton_cb(3, src, alpha=a)
    assert res.knife_edges == 0
    assert res.min_gap == abs((a + 0.0025) - a)
