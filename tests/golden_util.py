"""Loading and comparing the stored oracle outputs in tests/golden/.

The files are written by tests/golden/make_golden.py, which calls only the
oracle and the synthetic-input generator.
"""

import gzip
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(k: int):
    with gzip.open(os.path.join(GOLDEN, f"cfg{k}.json.gz"), "rt") as f:
        return json.load(f)


def expand(entry):
    """(adj, depth, sepsets) arrays/dict of one golden dataset entry."""
    n = entry["n_vars"]
    adj = np.zeros((n, n), dtype=np.uint8)
    for i, j in entry["kept_edges"]:
        adj[i, j] = adj[j, i] = 1
    depth = np.full((n, n), -1, dtype=np.int32)
    sep = {}
    for i, j, d, S in entry["removals"]:
        depth[i, j] = depth[j, i] = d
        sep[(i, j)] = tuple(S)
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j] and depth[i, j] < 0:
                depth[i, j] = depth[j, i] = 0
                sep[(i, j)] = ()
    return adj, depth, sep


def first_sepset_difference(got, want):
    """The first pair (in (i, j) order) whose separating set differs, with both."""
    for key in sorted(set(got) | set(want)):
        a, b = got.get(key), want.get(key)
        if a != b:
            n_diff = sum(1 for k in set(got) | set(want) if got.get(k) != want.get(k))
            return f"first at pair {key}: got {a}, oracle {b} ({n_diff} pair(s) differ)"
    return "no difference"


def compare_skeleton(got, entry, label=""):
    """Asserts identical skeleton, removal depths and sepsets, and that the
    per-depth canonical test counts equal the oracle's."""
    adj, depth, sep = expand(entry)
    assert got.adj.shape == adj.shape, label
    diff = np.argwhere(got.adj != adj)
    assert diff.size == 0, (f"{label}: skeleton differs at {diff[:5].tolist()}; "
                            f"sepsets: {first_sepset_difference(got.sepsets, sep)}")
    ddiff = np.argwhere(got.depth != depth)
    assert ddiff.size == 0, (f"{label}: removal depth differs at {ddiff[:5].tolist()}; "
                             f"sepsets: {first_sepset_difference(got.sepsets, sep)}")
    if got.sepsets != sep:
        raise AssertionError(f"{label}: sepsets differ: {first_sepset_difference(got.sepsets, sep)}")
    req = [s["tests_required"] for s in got.stats]
    assert req == entry["tests_per_depth"], f"{label}: tests per depth {req} vs {entry['tests_per_depth']}"
    rem = [s["removed"] for s in got.stats]
    assert rem == entry["removed_per_depth"], f"{label}: removed per depth {rem} vs {entry['removed_per_depth']}"


def compare_with_oracle(got, ref, label=""):
    """Asserts identical skeleton, removal depths, sepsets and per-depth
    canonical test and removal counts against a live oracle result."""
    diff = np.argwhere(got.adj != ref.adj)
    assert diff.size == 0, (f"{label}: skeleton differs at {diff[:5].tolist()}; "
                            f"sepsets: {first_sepset_difference(got.sepsets, ref.sepsets)}")
    ddiff = np.argwhere(got.depth != ref.depth)
    assert ddiff.size == 0, f"{label}: removal depth differs at {ddiff[:5].tolist()}"
    if got.sepsets != ref.sepsets:
        raise AssertionError(f"{label}: sepsets differ: {first_sepset_difference(got.sepsets, ref.sepsets)}")
    req = [s["tests_required"] for s in got.stats]
    assert req == ref.tests, f"{label}: tests per depth {req} vs {ref.tests}"
    rem = [s["removed"] for s in got.stats]
    assert rem == ref.removed, f"{label}: removed per depth {rem} vs {ref.removed}"
