"""Host-side logic of bench.py (no GPU): the one-GPU contract and the guard on
the committed HBM-traffic and L2 hit-rate figures."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_traffic_figure_follows_the_kernel_digest(tmp_path, monkeypatch):
    import bench
    # a workload without a counter summary has no traffic figure
    assert bench.measured_traffic("no_such_workload") is None
    # a summary is used only while its digest matches the device sources
    prof = tmp_path / "profiles"
    prof.mkdir()
    good = bench.kernel_sources_sha256()
    rec = dict(kernel="k_depth_tests", workload="w", hbm_bytes_per_launch=123.0,
               kernel_sources_sha256=good)
    (prof / "k_depth_tests_w_counters.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: good)
    assert bench.measured_traffic("w") == pytest.approx(123.0)
    rec["kernel_sources_sha256"] = "0" * 64
    (prof / "k_depth_tests_w_counters.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("w") is None


def test_committed_counter_summaries_are_well_formed():
    d = os.path.join(ROOT, "profiles")
    names = [n for n in os.listdir(d) if n.endswith("_counters.json")]
    assert names, "no committed counter summaries"
    for n in names:
        with open(os.path.join(d, n)) as f:
            rec = json.load(f)
        assert rec["kernel"] == "k_depth_tests"
        assert rec["hbm_bytes_per_launch"] > 0
        assert len(rec["kernel_sources_sha256"]) == 64
        # L2 hit rates (a separate counter run), when present, are fractions
        for p in rec["per_depth"]:
            if p.get("l2_hit_rate") is not None:
                assert 0.0 <= p["l2_hit_rate"] <= 1.0
                assert "l2_hit" in rec["commands"]


def test_l2_hit_rates_follow_the_kernel_digest(tmp_path, monkeypatch):
    import bench
    assert bench.measured_l2_hit_rates("no_such_workload") is None
    prof = tmp_path / "profiles"
    prof.mkdir()
    good = bench.kernel_sources_sha256()
    rec = dict(kernel="k_depth_tests", workload="w", hbm_bytes_per_launch=1.0, kernel_sources_sha256=good,
               per_depth=[dict(depth=0, l2_hit_rate=0.5), dict(depth=1, l2_hit_rate=0.25)])
    (prof / "k_depth_tests_w_counters.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: good)
    assert bench.measured_l2_hit_rates("w") == [0.5, 0.25]
    rec["kernel_sources_sha256"] = "0" * 64
    (prof / "k_depth_tests_w_counters.json").write_text(json.dumps(rec))
    assert bench.measured_l2_hit_rates("w") is None


def test_oracle_baseline_of_a_batch_uses_worker_processes():
    # a batch of small datasets: one full pass over worker processes, and the
    # same total of tests as the oracle run in this process
    import bench
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import oracle
    from bnsynth import make_dataset
    dss = [make_dataset(8 + k, 10, 2, 2, 3, 0.5, 500, seed=9100 + k) for k in range(3)]
    for d in dss:
        d.alpha, d.max_depth = 0.05, -1
    r = bench.cpu_baseline(dss)
    assert r["kind"] == "oracle" and r["value"] > 0
    assert 1 <= r["cores"] <= 3
    tests = sum(int(sum(oracle.pc_skeleton(d.data, d.cards, 0.05, -1).tests)) for d in dss)
    assert "3 datasets" in r["sample"]
    assert tests > 0
