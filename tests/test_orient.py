"""Parity of the library's orientation (bns_skeleton_orient, PC steps 2-3 of
Section III-C; host code, no GPU) with the orientation oracle.

Skeletons and sepsets are handed to the library with bns_skeleton_create:
those of random DAGs under a d-separation CI source (where the result is the
DAG's essential graph), planted conflicts, and the stored oracle skeletons of
the five workloads.  Marks must be identical.
"""

import networkx as nx
import numpy as np
import pytest

from golden_util import expand, load_golden
from oracle.orient import orient


@pytest.fixture(scope="module")
def bns():
    import paper_2212_04259_amd as b
    b.load()
    return b


def _dsep_source(dag):
    def p(x, y, s):
        return 1.0 if nx.is_d_separator(dag, {x}, {y}, set(s)) else 0.0
    return p


@pytest.mark.parametrize("seed", range(30))
def test_random_dags_match_oracle(bns, orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 12))
    order = rng.permutation(n)
    dag = nx.DiGraph()
    dag.add_nodes_from(range(n))
    for b in range(n):
        for a in range(b):
            if rng.random() < 0.35:
                dag.add_edge(int(order[a]), int(order[b]))
    res = orc.pc_skeleton_cb(n, _dsep_source(dag), alpha=0.5)
    assert np.array_equal(bns.bns_orient(res.adj, res.sepsets), orient(res.adj, res.sepsets))


def test_conflicts_match_oracle(bns):
    adj = np.zeros((6, 6), dtype=np.uint8)
    for a, b in [(0, 2), (1, 2), (2, 3), (3, 4), (3, 5)]:
        adj[a, b] = adj[b, a] = 1
    sep = {(i, j): () for i in range(6) for j in range(i + 1, 6) if not adj[i, j]}
    sep[(0, 3)] = sep[(1, 3)] = (2,)
    sep[(2, 4)] = sep[(2, 5)] = (3,)
    got = bns.bns_orient(adj, sep)
    assert np.array_equal(got, orient(adj, sep))
    assert got[2, 3] == 2 and got[3, 2] == 2
    path = np.zeros((4, 4), dtype=np.uint8)
    for a, b in [(0, 1), (1, 2), (2, 3)]:
        path[a, b] = path[b, a] = 1
    sp = {(0, 2): (), (1, 3): (), (0, 3): (1,)}
    assert np.array_equal(bns.bns_orient(path, sp), orient(path, sp))


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_stored_workload_skeletons_match_oracle(bns, k):
    for i, entry in enumerate(load_golden(k)["datasets"]):
        if k == 5 and i % 8:
            continue  # every eighth dataset of the batch keeps the CPU suite short
        adj, _, sep = expand(entry)
        got = bns.bns_orient(adj, sep)
        want = orient(adj, sep)
        assert np.array_equal(got, want), f"cfg{k}[{i}]"
        # marks are consistent with the skeleton
        assert np.array_equal(got > 0, adj > 0)


def test_invalid_skeletons_rejected(bns):
    import ctypes
    L = bns.load()
    n = 3
    adj = np.zeros((n, n), np.uint8)
    adj[0, 1] = 1  # not symmetric
    depth = np.full((n, n), -1, np.int32)
    off = np.full((n, n), -1, np.int64)
    pool = np.zeros(1, np.int32)
    h = ctypes.c_void_p()
    vp = ctypes.c_void_p
    st = L.bns_skeleton_create(n, adj.ctypes.data_as(vp), depth.ctypes.data_as(vp), off.ctypes.data_as(vp),
                               pool.ctypes.data_as(vp), 0, ctypes.byref(h))
    assert st == 1
    # a removed pair whose sepset points outside the pool
    adj[0, 1] = 0
    depth[0, 2] = depth[2, 0] = 1
    off[0, 2] = off[2, 0] = 5
    st = L.bns_skeleton_create(n, adj.ctypes.data_as(vp), depth.ctypes.data_as(vp), off.ctypes.data_as(vp),
                               pool.ctypes.data_as(vp), 1, ctypes.byref(h))
    assert st == 1
