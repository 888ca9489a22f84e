"""The autotuner's persistent cache and its samples-per-block dimension.

A first process tunes the smallest workload and appends its choice to the
cache file; a second process with the same file returns the same options at
once, without trial searches.  Malformed lines already in the file are
skipped.  Searches with the chosen options still match the oracle.
"""

import json
import os
import subprocess
import sys
import time

import pytest

from bnsynth import make_config
from golden_util import compare_skeleton, load_golden

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FIELDS = ("test_group", "max_replicas", "lds_bytes", "tickets_per_grab", "wave_depths",
          "block_depths", "split_min_samples", "units_per_group", "depth0", "round_tests", "depth1", "group_tests")

CHILD = r"""
import json, sys, time
sys.path.insert(0, {root!r}); sys.path.insert(0, {root!r} + "/tests")
import paper_2212_04259_amd as bns
from bnsynth import make_config
bns.load()
ds = make_config(1)[0]
h = bns.bns_dataset_create(ds.data, ds.cards)
t0 = time.perf_counter()
best = bns.bns_autotune([h], [ds.alpha], [ds.max_depth], trials=1)
dt = time.perf_counter() - t0
print("RESULT " + json.dumps({{"sec": dt, **{{f: int(getattr(best, f)) for f in {fields!r}}}}}), flush=True)
"""


def _child(cache):
    env = dict(os.environ, BNS_TUNE_CACHE=str(cache))
    code = CHILD.format(root=ROOT, fields=FIELDS)
    print(f"autotune child with cache {cache}", flush=True)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    line = [x for x in r.stdout.splitlines() if x.startswith("RESULT ")][-1]
    return json.loads(line[len("RESULT "):])


def test_cache_file_is_shared_between_processes(tmp_path):
    cache = tmp_path / "tune.txt"
    cache.write_text("not a tuning line\nbns4 gfx950/256cu 1,2,3 4 5\nbns4\n")
    first = _child(cache)
    lines = [x for x in cache.read_text().splitlines() if x.startswith("bns4 gfx950")]
    assert len(lines) == 2, cache.read_text()  # the malformed one and the new entry
    assert first["split_min_samples"] in (0, 2048, 8192, 16384, -1)
    assert first["units_per_group"] in (0, 4, 16)
    assert first["depth0"] in (0, 1, 2) and first["depth1"] in (0, 2)
    second = _child(cache)
    assert second["sec"] < 0.05, second
    assert {f: second[f] for f in FIELDS} == {f: first[f] for f in FIELDS}
    # nothing new appended by a cache hit
    assert cache.read_text().count("\n") == 4


def test_tuned_options_keep_results(tmp_path, monkeypatch):
    import paper_2212_04259_amd as bns
    bns.load()
    g = load_golden(1)["datasets"][0]
    ds = make_config(1)[0]
    h = bns.bns_dataset_create(ds.data, ds.cards)
    print("autotune cfg1 (fixed replication cap) in process", flush=True)
    base = bns.bns_options_default(max_replicas=16)
    best = bns.bns_autotune([h], [ds.alpha], [ds.max_depth], base, trials=1)
    assert best.max_replicas == 16  # what base fixes stays
    t0 = time.perf_counter()
    again = bns.bns_autotune([h], [ds.alpha], [ds.max_depth], base, trials=1)
    assert time.perf_counter() - t0 < 0.05
    assert all(getattr(again, f) == getattr(best, f) for f in FIELDS)
    got = bns.bns_pc_skeleton_dataset(h, ds.alpha, ds.max_depth, best)
    compare_skeleton(got, g, "cfg1 autotuned, replication cap fixed")
    for sm in (2048, -1):
        o = bns.bns_options_default(split_min_samples=sm, units_per_group=4)
        print(f"cfg1 split_min_samples={sm}", flush=True)
        sk = bns.bns_pc_skeleton_dataset(h, ds.alpha, ds.max_depth, o)
        compare_skeleton(sk, g, f"cfg1 split_min_samples={sm}")
        # the launch shape each depth ran with
        for s in sk.stats:
            assert s["test_group"] in (1, 2, 3), s
            if s["test_group"] == 3:
                assert s["depth"] == 0 and s["chunks"] == 0 and s["chunk_samples"] > 0
                continue
            assert s["chunks"] >= 1
            assert s["chunks"] * s["chunk_samples"] >= ds.n_samples
            if s["chunks"] > 1:
                assert sm > 0 and s["chunk_samples"] >= sm and s["chunk_samples"] % 1024 == 0
                assert (s["chunks"] - 1) * s["chunk_samples"] < ds.n_samples
            else:
                assert s["chunk_samples"] == ds.n_samples
        if sm == 2048:
            assert any(s["chunks"] > 1 for s in sk.stats), "cfg1's last depths have few tests: split"
