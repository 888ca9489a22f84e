"""Pins of the orientation oracle (PC steps 2 and 3 of Section III-C).

- Brute force: with a d-separation CI source the skeleton and sepsets of a
  DAG are exact, and steps 2-3 must return the DAG's essential graph.  That
  graph is computed here without any orientation rule: every orientation of
  the skeleton's edges is enumerated, the acyclic ones with the same
  v-structures as the DAG (its Markov equivalence class, Verma and Pearl) are
  kept, and an edge is directed iff all of them agree on its direction.
- Textbook graphs with hand-written CPDAGs (collider, chain, fork, diamond,
  a v-structure followed by R1, R2 and R3 configurations).
- A planted conflict: two v-structures orienting one edge both ways.
- Relabelling the variables relabels the result (no order dependence).
"""

import importlib.util
import itertools
import os

import networkx as nx
import numpy as np
import pytest


def _load_orient():
    # BNS_ORIENT_SRC points the pins at another copy of the orientation oracle
    # (the mutation suite runs them against deliberately broken copies)
    path = os.environ.get("BNS_ORIENT_SRC")
    if not path:
        from oracle.orient import orient as f
        return f
    spec = importlib.util.spec_from_file_location("orient_under_test", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.orient


orient = _load_orient()


def _dsep_source(dag):
    def p(x, y, s):
        return 1.0 if nx.is_d_separator(dag, {x}, {y}, set(s)) else 0.0
    return p


def _random_dag(rng, n, max_edges):
    order = rng.permutation(n)
    pairs = [(int(order[a]), int(order[b])) for a in range(n) for b in range(a + 1, n)]
    rng.shuffle(pairs)
    g = nx.DiGraph()
    g.add_nodes_from(range(n))
    for (u, v) in pairs[: int(rng.integers(1, max_edges + 1))]:
        g.add_edge(u, v)
    return g


def _v_structures(dag):
    out = set()
    for z in dag.nodes:
        ps = sorted(dag.predecessors(z))
        for a, b in itertools.combinations(ps, 2):
            if not dag.has_edge(a, b) and not dag.has_edge(b, a):
                out.add((a, z, b))
    return out


def _essential_graph(dag):
    """Marks of the essential graph by enumeration of the equivalence class."""
    n = dag.number_of_nodes()
    edges = sorted((min(u, v), max(u, v)) for u, v in dag.edges)
    vs = _v_structures(dag)
    members = []
    for bits in itertools.product((0, 1), repeat=len(edges)):
        g = nx.DiGraph()
        g.add_nodes_from(range(n))
        for (u, v), b in zip(edges, bits):
            g.add_edge(u, v) if b == 0 else g.add_edge(v, u)
        if nx.is_directed_acyclic_graph(g) and _v_structures(g) == vs:
            members.append(g)
    G = np.zeros((n, n), dtype=np.int8)
    for (u, v) in edges:
        fwd = all(g.has_edge(u, v) for g in members)
        bwd = all(g.has_edge(v, u) for g in members)
        G[u, v] = 2 if fwd else 1
        G[v, u] = 2 if bwd else 1
    return G, len(members)


def _pc_of(orc, dag):
    n = dag.number_of_nodes()
    res = orc.pc_skeleton_cb(n, _dsep_source(dag), alpha=0.5)
    return res.adj, res.sepsets


@pytest.mark.parametrize("seed", range(40))
def test_random_dags_give_their_essential_graph(orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 8))
    dag = _random_dag(rng, n, min(10, n * (n - 1) // 2))
    adj, sep = _pc_of(orc, dag)
    want, k = _essential_graph(dag)
    assert k >= 1
    got = orient(adj, sep)
    assert np.array_equal(got, want), (sorted(dag.edges), got.tolist(), want.tolist())


def _dag(edges, n):
    g = nx.DiGraph()
    g.add_nodes_from(range(n))
    g.add_edges_from(edges)
    return g


def _marks(n, directed=(), undirected=()):
    G = np.zeros((n, n), dtype=np.int8)
    for a, b in directed:
        G[a, b], G[b, a] = 2, 1
    for a, b in undirected:
        G[a, b] = G[b, a] = 1
    return G


@pytest.mark.parametrize("name,n,edges,directed,undirected", [
    ("collider", 3, [(0, 2), (1, 2)], [(0, 2), (1, 2)], []),
    ("chain", 3, [(0, 1), (1, 2)], [], [(0, 1), (1, 2)]),
    ("fork", 3, [(1, 0), (1, 2)], [], [(0, 1), (1, 2)]),
    ("diamond", 4, [(0, 1), (0, 2), (1, 3), (2, 3)], [(1, 3), (2, 3)], [(0, 1), (0, 2)]),
    # v-structure 0 -> 2 <- 1, then R1: 2 - 3 with 0, 3 not adjacent => 2 -> 3
    ("collider_then_R1", 4, [(0, 2), (1, 2), (2, 3)], [(0, 2), (1, 2), (2, 3)], []),
    # R2: 0 -> 2 <- 1 (v-structure), 2 -> 3 (R1), and 0 - 3 with 0 -> 2 -> 3 => 0 -> 3
    ("R2", 4, [(0, 2), (1, 2), (2, 3), (0, 3)], [(0, 2), (1, 2), (2, 3), (0, 3)], []),
    # R3: 1 -> 3 <- 2 (1, 2 not adjacent), 0 adjacent to 1, 2, 3 => 0 -> 3
    ("R3", 4, [(0, 1), (0, 2), (1, 3), (2, 3), (0, 3)], [(1, 3), (2, 3), (0, 3)], [(0, 1), (0, 2)]),
])
def test_textbook_graphs(orc, name, n, edges, directed, undirected):
    dag = _dag(edges, n)
    adj, sep = _pc_of(orc, dag)
    want = _marks(n, directed, undirected)
    assert np.array_equal(orient(adj, sep), want), name
    assert np.array_equal(_essential_graph(dag)[0], want), name


def test_planted_conflict_gets_two_arrowheads():
    # path 0 - 1 - 2 - 3 with empty sepsets: triple (0, 1, 2) orients
    # 0 -> 1 <- 2 and triple (1, 2, 3) orients 1 -> 2 <- 3: edge 1 - 2 conflicts
    adj = np.zeros((4, 4), dtype=np.uint8)
    for a, b in [(0, 1), (1, 2), (2, 3)]:
        adj[a, b] = adj[b, a] = 1
    sep = {(0, 2): (), (1, 3): (), (0, 3): (1,)}
    G = orient(adj, sep)
    assert G[0, 1] == 2 and G[1, 0] == 1
    assert G[1, 2] == 2 and G[2, 1] == 2
    assert G[3, 2] == 2 and G[2, 3] == 1


def test_sepset_membership_decides(orc):
    # the same skeleton with z inside or outside the sepset of (x, y)
    adj = np.zeros((3, 3), dtype=np.uint8)
    adj[0, 2] = adj[2, 0] = adj[1, 2] = adj[2, 1] = 1
    assert np.array_equal(orient(adj, {(0, 1): (2,)}), _marks(3, undirected=[(0, 2), (1, 2)]))
    assert np.array_equal(orient(adj, {(0, 1): ()}), _marks(3, directed=[(0, 2), (1, 2)]))


@pytest.mark.parametrize("seed", range(10))
def test_relabelling_relabels_the_result(orc, seed):
    rng = np.random.default_rng(100 + seed)
    n = 7
    dag = _random_dag(rng, n, 11)
    adj, sep = _pc_of(orc, dag)
    G = orient(adj, sep)
    perm = rng.permutation(n)
    dag2 = nx.relabel_nodes(dag, {i: int(perm[i]) for i in range(n)})
    adj2, sep2 = _pc_of(orc, dag2)
    G2 = orient(adj2, sep2)
    assert np.array_equal(G2[np.ix_(perm, perm)], G)


def test_meek_round_conflict_gets_two_arrowheads():
    # colliders 0 -> 2 <- 1 and 4 -> 3 <- 5 joined by the undirected edge 2 - 3:
    # in the first round R1 orients 2 -> 3 (from 0 -> 2, 0 and 3 not adjacent)
    # and 3 -> 2 (from 4 -> 3, 4 and 2 not adjacent) together
    adj = np.zeros((6, 6), dtype=np.uint8)
    for a, b in [(0, 2), (1, 2), (2, 3), (3, 4), (3, 5)]:
        adj[a, b] = adj[b, a] = 1
    sep = {(i, j): () for i in range(6) for j in range(i + 1, 6) if not adj[i, j]}
    sep[(0, 3)] = sep[(1, 3)] = (2,)
    sep[(2, 4)] = sep[(2, 5)] = (3,)
    G = orient(adj, sep)
    assert G[0, 2] == 2 and G[2, 0] == 1 and G[1, 2] == 2 and G[2, 1] == 1
    assert G[4, 3] == 2 and G[3, 4] == 1 and G[5, 3] == 2 and G[3, 5] == 1
    assert G[2, 3] == 2 and G[3, 2] == 2
