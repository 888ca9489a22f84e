"""Write the oracle's PC-stable results for the five synthetic workloads.

Calls only the oracle and the synthetic-input generator.  Output per config:
``tests/golden/cfg<k>.json.gz`` holding, per dataset, its sha256, the tests and
removals per depth, the final skeleton and every removal at depth >= 1 with
its sepset (pairs absent from both lists were removed at depth 0 with the
empty set).

    python tests/golden/make_golden.py 1 2 3        # configs to (re)write
    python tests/golden/make_golden.py 5 --jobs 6   # datasets in parallel
"""

import argparse
import gzip
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from bnsynth import make_config  # noqa: E402
from bnsynth.generate import CONFIGS, config_sizes, make_dataset  # noqa: E402


def summarize(ds, res, seconds):
    n = ds.n_vars
    kept = [[i, j] for i in range(n) for j in range(i + 1, n) if res.adj[i, j]]
    removals = [[i, j, int(res.depth[i, j]), list(S)] for (i, j), S in sorted(res.sepsets.items())
                if res.depth[i, j] >= 1]
    return dict(name=ds.name, sha256=ds.sha256(), n_vars=n, n_samples=ds.n_samples,
                alpha=ds.alpha, max_depth=ds.max_depth, tests_per_depth=res.tests,
                removed_per_depth=res.removed, knife_edges=res.knife_edges, min_gap=res.min_gap,
                kept_edges=kept, removals=removals, oracle_seconds=seconds)


def run_one(args):
    k, idx = args
    if "batch" in CONFIGS[k]:
        c = CONFIGS[k]
        n, m, seed = config_sizes(k)[idx]
        ds = make_dataset(n, int(round(c["edge_ratio"] * n)), c["max_indeg"], c["card_lo"],
                          c["card_hi"], c["dirichlet_alpha"], m, seed, c["alpha"], c["max_depth"],
                          f"{c['name']}[{idx}]")
    else:
        ds = make_config(k)[0]
    t0 = time.time()
    res = oracle.pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth)
    dt = time.time() - t0
    print(f"cfg{k}[{idx}] n={ds.n_vars} m={ds.n_samples} tests={sum(res.tests)} {dt:.1f}s", flush=True)
    return summarize(ds, res, dt)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("configs", nargs="+", type=int)
    ap.add_argument("--jobs", type=int, default=1)
    a = ap.parse_args()
    oracle.lib()
    for k in a.configs:
        n_ds = CONFIGS[k].get("batch", 1)
        jobs = [(k, i) for i in range(n_ds)]
        if a.jobs > 1 and n_ds > 1:
            with ProcessPoolExecutor(a.jobs) as ex:
                out = list(ex.map(run_one, jobs))
        else:
            out = [run_one(j) for j in jobs]
        path = os.path.join(HERE, f"cfg{k}.json.gz")
        with gzip.open(path, "wt") as f:
            json.dump(dict(config=k, datasets=out), f, separators=(",", ":"))
        print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
