"""Seeded generator of discrete Bayesian networks and their samples.

A network is drawn as follows, every random number coming from one
``numpy.random.Generator(PCG64(seed))`` in this fixed order:

1. a topological order: ``rng.permutation(n)``;
2. directed edges: two distinct positions of that order are drawn uniformly,
   the earlier one becomes the parent; the edge is kept when it is new and the
   child still has fewer than ``max_indeg`` parents; repeated until the target
   edge count is reached;
3. cardinalities: ``rng.integers(card_lo, card_hi + 1, n)``;
4. one CPT row per parent configuration, for variables 0..n-1 in id order,
   each row ~ Dirichlet(dirichlet_alpha * 1); parents are sorted ascending and
   the configuration index is mixed radix with the first parent fastest;
5. forward sampling in topological order, one ``rng.random(m)`` draw per
   variable turned into a category by the inverse CDF of its CPT row
   (clipped to card-1 against cumulative-sum rounding).

The joint distribution sampled is the BN factorisation of Section III-A: each
variable is drawn from P(V_i | Pa(V_i)) given its already-drawn parents.

Rows are stored ``uint8[n][m]``, C-contiguous: variable v's m samples are
contiguous (the paper's transposed, cache-friendly storage, Section IV-C).
"""

from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

# The five workloads.  Network sizes mirror the benchmark networks of Table II
# (Alarm/Insurance, Hepar2, Munin1, Munin2/3 scale); sample counts extend the
# paper's 5,000-15,000 rows to 50,000-200,000.
CONFIGS = {
    1: dict(name="cfg1_n20_m5k", n=20, edges=25, max_indeg=3, card_lo=2, card_hi=4,
            dirichlet_alpha=1.0, m=5_000, alpha=0.05, max_depth=-1, seed=101),
    2: dict(name="cfg2_n60_m50k", n=60, edges=70, max_indeg=4, card_lo=2, card_hi=4,
            dirichlet_alpha=0.5, m=50_000, alpha=0.05, max_depth=-1, seed=202),
    3: dict(name="cfg3_n220_m100k", n=220, edges=330, max_indeg=4, card_lo=2, card_hi=5,
            dirichlet_alpha=0.5, m=100_000, alpha=0.05, max_depth=-1, seed=303),
    4: dict(name="cfg4_n1000_m200k", n=1000, edges=1200, max_indeg=3, card_lo=2, card_hi=4,
            dirichlet_alpha=0.5, m=200_000, alpha=0.05, max_depth=4, seed=404),
    # A batch of 64 independent datasets; sizes drawn from the master seed,
    # dataset k uses seed 505000 + k.
    5: dict(name="cfg5_64x_n20-200_m5k-100k", batch=64, n_lo=20, n_hi=200, edge_ratio=1.25,
            max_indeg=3, card_lo=2, card_hi=5, dirichlet_alpha=0.5, m_lo=5_000,
            m_hi=100_000, alpha=0.01, max_depth=-1, seed=505),
}


@dataclass
class Dataset:
    data: np.ndarray            # uint8 [n][m], C-contiguous
    cards: np.ndarray           # uint8 [n]
    edges: list                 # true DAG edges (parent, child)
    alpha: float = 0.05
    max_depth: int = -1
    name: str = ""
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n_vars(self) -> int:
        return int(self.data.shape[0])

    @property
    def n_samples(self) -> int:
        return int(self.data.shape[1])

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.data.shape[0]).tobytes())
        h.update(np.int64(self.data.shape[1]).tobytes())
        h.update(np.ascontiguousarray(self.cards, dtype=np.uint8).tobytes())
        h.update(np.ascontiguousarray(self.data, dtype=np.uint8).tobytes())
        return h.hexdigest()

    def true_skeleton(self) -> np.ndarray:
        n = self.n_vars
        a = np.zeros((n, n), dtype=np.uint8)
        for p, c in self.edges:
            a[p, c] = a[c, p] = 1
        return a


def random_dag(rng: np.random.Generator, n: int, n_edges: int, max_indeg: int):
    """Steps 1-2: topological order and a set of (parent, child) edges."""
    order = rng.permutation(n)
    max_possible = sum(min(k, max_indeg) for k in range(n))
    target = min(n_edges, max_possible)
    present = set()
    indeg = np.zeros(n, dtype=np.int64)
    edges = []
    attempts = 0
    while len(edges) < target and attempts < 200 * max(target, 1) + 1000:
        attempts += 1
        a, b = rng.choice(n, size=2, replace=False)
        pa, pb = (a, b) if a < b else (b, a)
        parent, child = int(order[pa]), int(order[pb])
        if (parent, child) in present or indeg[child] >= max_indeg:
            continue
        present.add((parent, child))
        indeg[child] += 1
        edges.append((parent, child))
    return order, edges


def _parents_of(n: int, edges):
    parents = [[] for _ in range(n)]
    for p, c in edges:
        parents[c].append(p)
    return [sorted(ps) for ps in parents]


def random_cpts(rng: np.random.Generator, cards: np.ndarray, parents, dirichlet_alpha: float):
    """Step 4: one Dirichlet row per parent configuration, variables in id order."""
    cpts = []
    for v in range(len(cards)):
        n_cfg = int(np.prod([int(cards[p]) for p in parents[v]], dtype=np.int64)) if parents[v] else 1
        r = int(cards[v])
        cpts.append(rng.dirichlet(np.full(r, dirichlet_alpha), size=n_cfg))
    return cpts


def forward_sample(rng: np.random.Generator, order, parents, cards, cpts, m: int) -> np.ndarray:
    """Step 5: draw m rows from the BN factorisation, returned as uint8 [n][m]."""
    n = len(cards)
    out = np.zeros((n, m), dtype=np.uint8)
    for v in order:
        v = int(v)
        cfg = np.zeros(m, dtype=np.int64)
        stride = 1
        for p in parents[v]:
            cfg += out[p].astype(np.int64) * stride
            stride *= int(cards[p])
        cum = np.cumsum(cpts[v], axis=1)
        u = rng.random(m)
        val = (u[:, None] >= cum[cfg]).sum(axis=1)
        np.minimum(val, int(cards[v]) - 1, out=val)
        out[v] = val.astype(np.uint8)
    return out


def make_dataset(n: int, n_edges: int, max_indeg: int, card_lo: int, card_hi: int,
                 dirichlet_alpha: float, m: int, seed: int, alpha: float = 0.05,
                 max_depth: int = -1, name: str = "") -> Dataset:
    rng = np.random.Generator(np.random.PCG64(seed))
    order, edges = random_dag(rng, n, n_edges, max_indeg)
    cards = rng.integers(card_lo, card_hi + 1, n).astype(np.uint8)
    parents = _parents_of(n, edges)
    cpts = random_cpts(rng, cards, parents, dirichlet_alpha)
    data = forward_sample(rng, order, parents, cards, cpts, m)
    return Dataset(data=np.ascontiguousarray(data), cards=cards, edges=edges, alpha=alpha,
                   max_depth=max_depth, name=name, seed=seed,
                   meta=dict(n=n, edges=len(edges), max_indeg=max_indeg, card_lo=card_lo,
                             card_hi=card_hi, dirichlet_alpha=dirichlet_alpha, m=m))


def config_sizes(k: int):
    """Per-dataset (n, m, seed) of a config, without sampling any rows."""
    c = CONFIGS[k]
    if "batch" not in c:
        return [(c["n"], c["m"], c["seed"])]
    rng = np.random.Generator(np.random.PCG64(c["seed"]))
    ns = rng.integers(c["n_lo"], c["n_hi"] + 1, c["batch"])
    ms = rng.integers(c["m_lo"], c["m_hi"] + 1, c["batch"])
    return [(int(ns[i]), int(ms[i]), c["seed"] * 1000 + i) for i in range(c["batch"])]


def make_config(k: int, m_override: int | None = None):
    """Datasets of config k (a list; one element except for the batched config)."""
    c = CONFIGS[k]
    out = []
    if "batch" not in c:
        m = c["m"] if m_override is None else m_override
        out.append(make_dataset(c["n"], c["edges"], c["max_indeg"], c["card_lo"], c["card_hi"],
                                c["dirichlet_alpha"], m, c["seed"], c["alpha"], c["max_depth"],
                                c["name"]))
        return out
    for i, (n, m, seed) in enumerate(config_sizes(k)):
        if m_override is not None:
            m = m_override
        out.append(make_dataset(n, int(round(c["edge_ratio"] * n)), c["max_indeg"], c["card_lo"],
                                c["card_hi"], c["dirichlet_alpha"], m, seed, c["alpha"],
                                c["max_depth"], f"{c['name']}[{i}]"))
    return out
