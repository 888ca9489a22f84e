"""Benchmark: batched G^2 CI tests of PC-stable skeleton learning on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 2]

A step is one complete skeleton search (every depth of Algorithm 1: queue
build, all CI tests, removals) over one synthetic dataset already resident in
device memory.  The default workload is the 60-variable, 50,000-row network
(the configuration the plain-versus-batched metric is quoted on).  Prints one
JSON line; ``value`` is CI tests per second, counting the tests of the
sequential order (per edge, up to and including its first accepting test).
After timing, one of the timed searches is compared with the stored oracle
results of the workload (skeleton, removal depths, sepsets, per-depth test
counts); a mismatch sets ``parity`` false and the exit status to 1.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TIMING_SEARCHES = 5
# Integer vector ALU of MI355X: 256 compute units, 4 SIMDs of 16 lanes each
# (a wave64 instruction occupies a SIMD for 4 cycles), 2.4 GHz peak clock.
ALU_LANE_OPS_PER_S = 256 * 64 * 2.4e9


def _sum(stats, key):
    return sum(s[key] for s in stats)


def depth_totals(sks):
    """Per-depth counters of a search over all its problems: each handle of a
    multi-dataset search holds its own problem's counters (up to its last
    depth with a test); the launch timings are shared."""
    n = max(len(sk.stats) for sk in sks)
    out = []
    for d in range(n):
        rows = [sk.stats[d] for sk in sks if d < len(sk.stats)]
        t = {k: sum(r[k] for r in rows) for k in ("edges", "tests_required", "tests_executed", "removed",
                                                   "rechecks", "tickets", "operand_bytes")}
        t["depth"] = d
        t["span_seconds"] = rows[0]["span_seconds"]
        t["kernel_seconds"] = rows[0]["kernel_seconds"]
        for k in ("test_group", "chunks", "chunk_samples"):  # launch shape, shared
            t[k] = rows[0].get(k, 0)
        out.append(t)
    return out


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def _oracle_search(args):
    """One dataset's search by the oracle in a worker process: its tests."""
    import oracle
    data, cards, alpha, max_depth = args
    r = oracle.pc_skeleton(data, cards, alpha, max_depth)
    return int(sum(r.tests))


def _oracle_ready(_):
    import oracle
    oracle.lib()
    return 0


def cpu_baseline(datasets, budget_s=10.0):
    """The oracle on the same workload: a single thread repeated up to
    ~budget_s for one dataset; for a batch of independent datasets, one full
    run with one worker process per host core (at most 16), each worker
    running whole datasets one after another (the oracle itself is single
    threaded)."""
    if len(datasets) > 1:
        return _cpu_baseline_pool(datasets)
    import oracle
    oracle.lib()
    tests, t0, runs = 0, time.perf_counter(), 0
    while True:
        for ds in datasets:
            r = oracle.pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth)
            tests += sum(r.tests)
        runs += 1
        el = time.perf_counter() - t0
        if el >= budget_s or runs >= 50:
            break
    model, avail = host_cpu()
    return dict(value=tests / el, unit="CI tests/s", cores=1, kind="oracle",
                sample=f"{runs} full run(s) of the workload, single thread, {el:.1f} s",
                cpu_model=model, host_cpus_available=avail)


def _cpu_baseline_pool(datasets):
    import multiprocessing as mp
    model, avail = host_cpu()
    workers = max(1, min(len(datasets), avail, 16))
    # fresh interpreters (the parent has initialised the GPU: no fork of it)
    ctx = mp.get_context("spawn")
    args = [(d.data, d.cards, d.alpha, d.max_depth) for d in datasets]
    with ctx.Pool(workers) as pool:
        pool.map_async(_oracle_ready, range(workers)).get(timeout=300)
        t0 = time.perf_counter()
        tests = sum(pool.map_async(_oracle_search, args, chunksize=1).get(timeout=1800))
        el = time.perf_counter() - t0
    return dict(value=tests / el, unit="CI tests/s", cores=workers, kind="oracle",
                sample=f"one full run of the {len(datasets)} datasets, {workers} worker processes "
                       f"(whole datasets each, data passed to the workers inside the timing), {el:.1f} s",
                cpu_model=model, host_cpus_available=avail)


def kernel_sources_sha256():
    """Digest of the device-code sources of the library (csrc/*.h and the
    kernels; the host-side C ABI in capi.hip does not change kernel traffic)."""
    import hashlib
    d = os.path.join(ROOT, "paper_2212_04259_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h")) and name != "capi.hip":
            h.update(name.encode())
            with open(os.path.join(d, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload):
    """Bytes per test launch that left L2 (rocprofv3 FETCH_SIZE + WRITE_SIZE,
    calibrated against a copy of known size) from the committed counter
    summary of this workload, or None when there is none or the kernels have
    changed since the counters were taken.  FETCH_SIZE counts L2 misses,
    which the Infinity Cache may still serve: an upper bound on DRAM bytes."""
    path = os.path.join(ROOT, "profiles", f"k_depth_tests_{workload}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    return rec.get("hbm_bytes_per_launch")


def measured_l2_hit_rates(workload):
    """Per-depth L2 hit rates (rocprofv3 TCC_HIT / (TCC_HIT + TCC_MISS)) from
    the committed counter summary of this workload, or None as for
    measured_traffic."""
    path = os.path.join(ROOT, "profiles", f"k_depth_tests_{workload}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    rates = [p.get("l2_hit_rate") for p in rec.get("per_depth", [])]
    return rates if any(r is not None for r in rates) else None


def streaming_read_peak_gbs(torch, gib=4, reps=10):
    """Device read bandwidth of this machine: float reductions (sum, max) over a
    buffer far larger than the last-level cache (GB/s, best of reps and of
    the two reductions)."""
    n = gib << 30
    x = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    best = 0.0
    for op in (torch.sum, torch.amax):
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            s = op(x)
            e1.record()
            e1.synchronize()
            best = max(best, n / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del s, x
    torch.cuda.empty_cache()
    return best


def precision_report(bns, handle, ds, per_depth=2000, seed=7):
    """FP32 G^2 (the default arithmetic) against FP64 on a seeded sample of
    tests of the workload: random (x, y, Z) with |Z| = 0..3 over its variables.
    The relative error covers the results the FP32 form reports without an
    FP64 re-check (recheck band 0, so only the propagated-bound re-checks
    remain); decisions are compared for every test."""
    import numpy as np
    rng = np.random.default_rng(seed)
    tests = []
    for d in range(4):
        for _ in range(per_depth):
            vs = rng.choice(ds.n_vars, size=d + 2, replace=False)
            tests.append((int(vs[0]), int(vs[1]), tuple(int(v) for v in vs[2:])))
    r32 = bns.bns_ci_batch(handle, tests, ds.alpha,
                           bns.bns_options_default(precision=0, recheck_band=0.0))
    r64 = bns.bns_ci_batch(handle, tests, ds.alpha, bns.bns_options_default(precision=1))
    raw = (r32["flags"] & 2) == 0
    rel = np.abs(r32["g2"] - r64["g2"]) / np.maximum(np.abs(r64["g2"]), 1.0)
    rr = rel[raw]
    return {
        "tests": len(tests),
        "conditioning_sizes": [0, 1, 2, 3],
        "g2_rel_err_max": float(rr.max()) if rr.size else 0.0,
        "g2_rel_err_p99": float(np.quantile(rr, 0.99)) if rr.size else 0.0,
        "g2_rel_err_median": float(np.median(rr)) if rr.size else 0.0,
        "rechecked_fraction": float(1.0 - raw.mean()),
        "decisions_equal_fp64": bool(np.array_equal(r32["flags"] & 1, r64["flags"] & 1)),
    }


def search_error_report(bns, handles, alphas, maxd, knobs):
    """The search's own tests in verification mode (every executed test also
    evaluated in FP64): FP32 relative error of G^2 per depth, untimed."""
    o = bns.bns_options_default(report_errors=1, **knobs)
    if len(handles) == 1:
        sks = [bns.bns_pc_skeleton_dataset(handles[0], alphas[0], maxd[0], o)]
    else:
        sks = bns.bns_pc_skeleton_batch(handles, alphas, maxd, o)
    per_depth = []
    for d in range(max(len(sk.stats) for sk in sks)):
        rows = [sk.stats[d] for sk in sks if d < len(sk.stats)]
        per_depth.append({"depth": d, "tests": sum(r["err_tests"] for r in rows),
                          "max": max(r["err_max"] for r in rows),
                          "p99_max_over_problems": max(r["err_p99"] for r in rows),
                          "p50_max_over_problems": max(r["err_p50"] for r in rows),
                          "fp32_only_flips": sum(r["err_flips"] for r in rows),
                          "rechecks": sum(r["rechecks"] for r in rows)})
    return {"tests": sum(p["tests"] for p in per_depth),
            "max": max(p["max"] for p in per_depth),
            "fp32_only_flips": sum(p["fp32_only_flips"] for p in per_depth),
            "per_depth": per_depth}


def check_parity(sks, config):
    """Compares a timed search's results with the stored oracle results of
    the workload (tests/golden); returns (ok, message)."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from golden_util import compare_skeleton, load_golden
    gold = load_golden(config)["datasets"]
    if len(gold) != len(sks):
        return False, f"{len(sks)} results against {len(gold)} stored"
    try:
        for i, (sk, g) in enumerate(zip(sks, gold)):
            compare_skeleton(sk, g, f"dataset {i}")
    except AssertionError as e:
        return False, str(e)
    return True, "identical to the oracle"


def study(bns, torch, handles, dss, alphas, maxd, config, steps, warmup, with_plain):
    """Granularity and level-width study (Sections IV-A and IV-B): the same
    workload through the sample-level form (plain, one sample-parallel launch
    per test), the edge-level form (one group per edge) and the CI-level
    batched form, then the batched form with levels of g ranks per edge.  Per
    row: ms per search (median of the timed searches), canonical CI tests per
    second, and the extra-tests proportion (executed / required - 1)."""
    import statistics

    def timed(o, n_steps, n_warm):
        def run():
            if len(handles) == 1:
                return [bns.skeleton_handle(handles[0], alphas[0], maxd[0], o)]
            return bns.skeleton_batch_handles(handles, alphas, maxd, o)
        for _ in range(n_warm):
            for h in run():
                bns.free_skeleton(h)
        torch.cuda.synchronize()
        ts, sks = [], None
        for _ in range(n_steps):
            t0 = time.perf_counter()
            hs = run()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            cur = [bns.collect(h) for h in hs]
            sks = sks or cur
        tot = depth_totals(sks)
        req, ex = _sum(tot, "tests_required"), _sum(tot, "tests_executed")
        ok, _ = check_parity(sks, config)
        ms = 1e3 * statistics.median(ts)
        return {"ms_per_search": ms, "ci_tests_per_s": req / (ms * 1e-3), "tests_required": req,
                "tests_executed": ex, "extra_tests": ex / req - 1.0, "parity": ok}

    rows = []
    forms = [("batched (CI-level)", dict()), ("edge-level, wave per edge", dict(form=bns.BNS_FORM_EDGE)),
             ("edge-level, workgroup per edge", dict(form=bns.BNS_FORM_EDGE, test_group=2))]
    if with_plain:
        forms.append(("plain (sample-level)", dict(form=bns.BNS_FORM_PLAIN, precision=1)))
    for name, kw in forms:
        plain = kw.get("form") == bns.BNS_FORM_PLAIN
        r = timed(bns.bns_options_default(**kw), 1 if plain else steps, 0 if plain else warmup)
        rows.append(dict(study="granularity", form=name, **r))
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    for g in (0, 1, 2, 4, 6, 8, 10, 16, 32):
        r = timed(bns.bns_options_default(round_tests=g), steps, warmup)
        rows.append(dict(study="level width", round_tests=g, **r))
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--precision", type=int, default=0, help="0 FP32+FP64 recheck, 1 FP64")
    ap.add_argument("--lds-bytes", type=int, default=0)
    ap.add_argument("--wg-per-cu", type=int, default=0)
    ap.add_argument("--split-min", type=int, default=0,
                    help="smallest sample chunk of split tests (0 default, -1 never split)")
    ap.add_argument("--units-per-group", type=int, default=0)
    ap.add_argument("--test-group", type=int, default=0, help="0 auto, 1 wave, 2 workgroup")
    ap.add_argument("--max-replicas", type=int, default=0)
    ap.add_argument("--tickets-per-grab", type=int, default=0)
    ap.add_argument("--wave-depths", type=int, default=0,
                    help="bit d set: one wave per test at depth d")
    ap.add_argument("--block-depths", type=int, default=0,
                    help="bit d set: one workgroup per test at depth d")
    ap.add_argument("--depth0", type=int, default=0, help="0 auto, 1 test kernel, 2 pair tables")
    ap.add_argument("--depth1", type=int, default=0, help="0 auto, 1 test kernel, 2 masked Gram tables")
    ap.add_argument("--group-tests", type=int, default=0,
                    help="depth 1 work units: 0 auto, 1 one test, 2 one edge's ranks of a level")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-stream-peak", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the given options instead of the autotuned ones")
    ap.add_argument("--study", action="store_true",
                    help="granularity (plain / edge-level / batched) and level-width study instead of the "
                         "benchmark line")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one device copy of this many MiB first (profiler byte calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {a.gpus}): the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2212_04259_amd as bns
    from bnsynth import make_config
    from bnsynth.generate import CONFIGS

    torch.cuda.set_device(0)
    if a.calib_copy_mb > 0:
        # Profiler byte calibration: one device copy of a known size whose
        # source has been pushed out of L2 and the Infinity Cache first (by
        # writing a 1 GiB buffer after it), so the copy reads it from HBM.
        n = a.calib_copy_mb << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        flush = torch.zeros(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst, flush
    dss = make_config(a.config)
    # Inputs resident in device memory before the timed region.
    handles = [bns.bns_dataset_create(d.data, d.cards) for d in dss]
    alphas = [d.alpha for d in dss]
    maxd = [d.max_depth for d in dss]
    if a.study:
        rows = study(bns, torch, handles, dss, alphas, maxd, a.config, a.steps, a.warmup,
                     with_plain=not a.no_plain and len(dss) == 1 and a.config <= 2)
        print(json.dumps({"workload": CONFIGS[a.config]["name"], "rows": rows}), flush=True)
        return
    knobs = dict(precision=a.precision, lds_bytes=a.lds_bytes, wg_per_cu=a.wg_per_cu,
                 split_min_samples=a.split_min, units_per_group=a.units_per_group,
                 test_group=a.test_group, max_replicas=a.max_replicas,
                 tickets_per_grab=a.tickets_per_grab, wave_depths=a.wave_depths,
                 block_depths=a.block_depths, depth0=a.depth0, depth1=a.depth1,
                 group_tests=a.group_tests)
    opt = bns.bns_options_default(**knobs)
    tuned = None
    if not a.no_autotune:
        # launch options chosen by the library's autotuner (untimed setup)
        opt = bns.bns_autotune(handles, alphas, maxd, opt)
        tuned = {f: getattr(opt, f) for f in ("test_group", "max_replicas", "lds_bytes",
                                               "tickets_per_grab", "wave_depths", "block_depths",
                                               "split_min_samples", "units_per_group", "depth0", "depth1",
                                               "group_tests")}
        knobs.update(tuned)

    def step(o):
        if len(handles) == 1:
            return [bns.skeleton_handle(handles[0], alphas[0], maxd[0], o)]
        return bns.skeleton_batch_handles(handles, alphas, maxd, o)

    for _ in range(a.warmup):
        for h in step(opt):
            bns.free_skeleton(h)
    torch.cuda.synchronize()
    kept = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        kept.append(step(opt))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = 1e3 * el / a.steps
    # test-kernel execution spans of the timed searches (device clock stamps,
    # per depth), and the results of the first timed search for the parity check
    spans = []
    first = None
    for hs in kept:
        sks = [bns.collect(h) for h in hs]
        if first is None:
            first = sks
        spans.append([t["span_seconds"] for t in depth_totals(sks)])
    ndep = min(len(s) for s in spans)
    span_d = [sum(s[d] for s in spans) / len(spans) for d in range(ndep)]
    span = sum(span_d)
    parity_ok, parity_msg = check_parity(first, a.config)

    # Counters of a few more (untimed) searches, with HIP events around each
    # depth's persistent test launch (on the launch stream); the event time
    # is the mean over these searches.
    topt = bns.bns_options_default(timing=1, **knobs)
    ksecs = []
    for _ in range(TIMING_SEARCHES):
        sks = [bns.collect(h) for h in step(topt)]
        tot = depth_totals(sks)
        ksecs.append(_sum(tot, "kernel_seconds"))
    required = _sum(tot, "tests_required")
    executed = _sum(tot, "tests_executed")
    rechecks = _sum(tot, "rechecks")
    obytes_exec = _sum(tot, "operand_bytes")
    ksec = sum(ksecs) / len(ksecs)
    m_of = [d.n_samples for d in dss]
    launches = len(tot)
    # Algorithmic work of the method's own (required) tests: a depth-d test
    # reads (d + 2) m operand bytes and does (d + 2) m int32 operations (d + 1
    # cell-index multiply-adds and one table increment per sample).  Per-problem
    # sample counts differ in a batch, so the required bytes come per problem.
    req_bytes_d = [0.0] * launches
    for sk, m in zip(first, m_of):
        for d, s in enumerate(sk.stats):
            req_bytes_d[d] += s["tests_required"] * (d + 2) * m
    req_bytes = sum(req_bytes_d)
    ops_rate = req_bytes / span if span > 0 else 0.0          # int32 ops/s (= required bytes/s)
    traffic = measured_traffic(CONFIGS[a.config]["name"])
    l2_hit = measured_l2_hit_rates(CONFIGS[a.config]["name"])
    # LDS increments of the counting step: one per sample of each executed
    # test (operand bytes / (d + 2) columns); the contraction paths count on
    # MFMA and have none.  Peak: this device's own rate (bns_lds_increment_rate).
    lds_peak = bns.bns_lds_increment_rate(0)[0]
    incs_d = [tot[d]["operand_bytes"] / (d + 2) if tot[d]["test_group"] != 3 else 0.0 for d in range(launches)]
    per_depth = []
    for d in range(min(launches, ndep)):
        sd = span_d[d]
        per_depth.append({
            "depth": d, "span_us": sd * 1e6, "tests_required": tot[d]["tests_required"],
            "tests_executed": tot[d]["tests_executed"],
            "alu_frac": (req_bytes_d[d] / sd) / ALU_LANE_OPS_PER_S if sd > 0 else None,
            "operand_gbs_required": req_bytes_d[d] / sd / 1e9 if sd > 0 else None,
            "lanes_per_test": {1: "wave", 2: "workgroup", 3: "Gram contraction"}.get(tot[d]["test_group"]),
            "chunks": tot[d]["chunks"], "chunk_samples": tot[d]["chunk_samples"],
            "lds_frac": (incs_d[d] / sd) / lds_peak if (lds_peak and sd > 0 and incs_d[d] > 0) else None,
        })
    count_span = sum(span_d[d] for d in range(min(launches, ndep)) if incs_d[d] > 0)
    lds_rate = sum(incs_d[:ndep]) / count_span if count_span > 0 else None
    stream_peak = None if a.no_stream_peak else streaming_read_peak_gbs(torch)

    out = {
        "metric": "CI tests/sec (batched, same skeleton as the FP64 oracle)",
        "value": required / (ms * 1e-3),
        "unit": "CI tests/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32 counts + f32 G2 + f64 p",
        "data": "synthetic",
        "config": {
            "workload": CONFIGS[a.config]["name"],
            "datasets": len(dss),
            "n_vars": [d.n_vars for d in dss] if len(dss) > 1 else dss[0].n_vars,
            "n_samples": sum(m_of),
            "alpha": alphas[0],
            "max_depth": maxd[0],
            "g2_arithmetic": "fp64" if a.precision == 1 else "fp32 + fp64 recheck",
            "form": "batched persistent per-depth launch",
            "autotuned": tuned,
        },
        "parity": parity_ok,
        "parity_detail": parity_msg,
        "tests_required_per_step": required,
        "tests_executed_per_step": executed,
        "waste_ratio": executed / required - 1.0 if required else 0.0,
        "recheck_fraction": rechecks / executed if executed else 0.0,
        "sample_rows_per_s": sum(s["tests_required"] * m for sk, m in zip(first, m_of) for s in sk.stats)
        / (ms * 1e-3),
        "depths": launches,
        # The test kernel's binding roof class: its operands are cache-resident
        # on this workload (DRAM traffic a few percent of the operand bytes),
        # so the roof it would meet with its per-test latency hidden is the
        # integer vector ALU of the counting loop.
        "roofline": {
            "bound": "alu",
            "kernel": "k_depth_tests",
            "achieved": ops_rate / 1e12,
            "peak": ALU_LANE_OPS_PER_S / 1e12,
            "unit": "T int32 ops/s",
            "frac": ops_rate / ALU_LANE_OPS_PER_S,
            "traffic": traffic,
            "basis": "(d+2) int32 ops per sample of each required depth-d test over the test "
                     "kernel's device-clock span; peak 256 CU x 64 lanes x 2.4 GHz",
            "launches": launches,
            "kernel_ms_per_step": span * 1e3,
            "kernel_ms_per_step_hip_events": ksec * 1e3,
            "per_depth": per_depth,
        },
        "hbm_roof": {
            "operand_gbs_required": req_bytes / span / 1e9 if span > 0 else None,
            "operand_gbs_executed": obytes_exec / span / 1e9 if span > 0 else None,
            "peak_gbs": HBM_PEAK_GBS,
            "frac_required": req_bytes / span / 1e9 / HBM_PEAK_GBS if span > 0 else None,
            "frac_executed": obytes_exec / span / 1e9 / HBM_PEAK_GBS if span > 0 else None,
            "operand_bytes_required_per_step": req_bytes,
            "operand_bytes_executed_per_step": obytes_exec,
            "l2_egress_bytes_per_launch": traffic,
            "l2_egress_gbs": (traffic / (span / launches) / 1e9) if (traffic and span > 0) else None,
            "l2_egress_frac_hbm": (traffic / (span / launches) / 1e9 / HBM_PEAK_GBS)
            if (traffic and span > 0) else None,
            "l2_hit_rate_per_depth": l2_hit,
            "streaming_read_peak_gbs": stream_peak,
            "frac_required_of_streaming_peak": (req_bytes / span / 1e9 / stream_peak)
            if (stream_peak and span > 0) else None,
        },
        # The counting step's own resource: one LDS increment per sample and
        # executed test, against the increment rate measured on this device.
        "lds_roof": {
            "achieved": lds_rate / 1e12 if lds_rate else None,
            "peak_measured": lds_peak / 1e12 if lds_peak else None,
            "unit": "T LDS increments/s",
            "frac": lds_rate / lds_peak if (lds_rate and lds_peak) else None,
            "basis": "one LDS increment per sample of each executed test over the spans of the depths "
                     "that count in LDS; peak: bns_lds_increment_rate on this device",
        },
    }

    if not a.no_plain and len(dss) == 1:
        popt = bns.bns_options_default(form=bns.BNS_FORM_PLAIN, precision=1)
        t0 = time.perf_counter()
        h = bns.skeleton_handle(handles[0], alphas[0], maxd[0], popt)
        torch.cuda.synchronize()
        pel = time.perf_counter() - t0
        psk = bns.collect(h)
        same = (psk.adj == first[0].adj).all() and psk.sepsets == first[0].sepsets
        preq = _sum(psk.stats, "tests_required")
        out["plain_form"] = {"value": preq / pel, "unit": "CI tests/s", "ms_per_step": pel * 1e3,
                             "same_skeleton_and_sepsets": bool(same)}
        out["speedup_vs_plain"] = out["value"] / out["plain_form"]["value"]

    if not a.no_precision:
        out["precision_fp32_vs_fp64"] = precision_report(bns, handles[0], dss[0])
        if a.precision == 0:
            out["search_fp32_error"] = search_error_report(bns, handles, alphas, maxd, knobs)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(dss)
    print(json.dumps(out), flush=True)
    if not parity_ok:
        print(f"parity failure: {parity_msg}", file=sys.stderr)
        sys.exit(1)


if __name__ == "__main__":
    main()
