"""Benchmark: batched G^2 CI tests of PC-stable skeleton learning on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 2]

A step is one complete skeleton search (every depth of Algorithm 1: queue
build, all CI tests, removals) over one synthetic dataset already resident in
device memory.  The default workload is the 60-variable, 50,000-row network
(the configuration the plain-versus-batched metric is quoted on).  Prints one
JSON line; ``value`` is CI tests per second, counting the tests of the
sequential order (per edge, up to and including its first accepting test).
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


def _sum(stats, key):
    return sum(s[key] for s in stats)


def _stats_of(bns, h):
    sk = bns.collect(h)
    return sk, sk.stats


def cpu_baseline(datasets, budget_s=10.0):
    """The oracle (single thread) on the same workload, repeated up to ~budget_s."""
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
    return dict(value=tests / el, unit="CI tests/s", cores=1, kind="oracle",
                sample=f"{runs} full run(s) of the workload, single thread, {el:.1f} s")


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
    """HBM bytes per test launch from the committed rocprofv3 counter summary
    of this workload (FETCH_SIZE + WRITE_SIZE, calibrated against a copy of
    known size), or None when there is none or the kernels have changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"k_depth_tests_{workload}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    return rec.get("hbm_bytes_per_launch")


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
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the given options instead of the autotuned ones")
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
    knobs = dict(precision=a.precision, lds_bytes=a.lds_bytes, wg_per_cu=a.wg_per_cu,
                 split_min_samples=a.split_min, units_per_group=a.units_per_group,
                 test_group=a.test_group, max_replicas=a.max_replicas,
                 tickets_per_grab=a.tickets_per_grab, wave_depths=a.wave_depths,
                 block_depths=a.block_depths)
    opt = bns.bns_options_default(**knobs)
    tuned = None
    if not a.no_autotune:
        # launch options chosen by the library's autotuner (untimed setup)
        opt = bns.bns_autotune(handles, alphas, maxd, opt)
        tuned = {f: getattr(opt, f) for f in ("test_group", "max_replicas", "lds_bytes",
                                               "tickets_per_grab", "wave_depths", "block_depths")}
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
    # test-kernel execution spans of the timed searches (device clock stamps)
    span = 0.0
    for hs in kept:
        sk0 = bns.collect(hs[0])
        span += _sum(sk0.stats, "span_seconds")
        for h in hs[1:]:
            bns.free_skeleton(h)
    span /= len(kept)

    # Counters of a few more (untimed) searches, with HIP events around each
    # depth's persistent test launch (on the launch stream) for the roofline
    # of that kernel; the kernel time is the mean over these searches.
    topt = bns.bns_options_default(timing=1, **knobs)
    ksecs = []
    for _ in range(TIMING_SEARCHES):
        hs = step(topt)
        sks = [bns.collect(h) for h in hs]
        ksecs.append(_sum(sks[0].stats, "kernel_seconds"))
    stats = sks[0].stats          # a multi-dataset search shares one set of counters
    required = _sum(stats, "tests_required")
    executed = _sum(stats, "tests_executed")
    rechecks = _sum(stats, "rechecks")
    obytes = _sum(stats, "operand_bytes")
    ksec = sum(ksecs) / len(ksecs)
    m_total = sum(d.n_samples for d in dss)
    rows_per_test = m_total / len(dss)
    launches = len(stats)
    # achieved: operand bytes per launch over the launch's execution span in
    # the timed searches
    achieved = (obytes / launches) / (span / launches) / 1e9 if span > 0 else None

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
        "dtype": "u8",
        "data": "synthetic",
        "config": {
            "workload": CONFIGS[a.config]["name"],
            "datasets": len(dss),
            "n_vars": [d.n_vars for d in dss] if len(dss) > 1 else dss[0].n_vars,
            "n_samples": m_total,
            "alpha": alphas[0],
            "max_depth": maxd[0],
            "g2_arithmetic": "fp64" if a.precision == 1 else "fp32 + fp64 recheck",
            "form": "batched persistent per-depth launch",
            "autotuned": tuned,
        },
        "tests_required_per_step": required,
        "tests_executed_per_step": executed,
        "waste_ratio": executed / required - 1.0 if required else 0.0,
        "recheck_fraction": rechecks / executed if executed else 0.0,
        "sample_rows_per_s": required * rows_per_test / (ms * 1e-3),
        "depths": launches,
        "roofline": {
            "bound": "hbm",
            "kernel": "k_depth_tests",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": measured_traffic(CONFIGS[a.config]["name"]),
            "launches": launches,
            "kernel_ms_per_step": span * 1e3,
            "kernel_ms_per_step_hip_events": ksec * 1e3,
            "operand_bytes_per_step": obytes,
        },
    }

    if not a.no_plain and len(dss) == 1:
        popt = bns.bns_options_default(form=bns.BNS_FORM_PLAIN, precision=1)
        t0 = time.perf_counter()
        h = bns.skeleton_handle(handles[0], alphas[0], maxd[0], popt)
        torch.cuda.synchronize()
        pel = time.perf_counter() - t0
        psk = bns.collect(h)
        same = (psk.adj == sks[0].adj).all() and psk.sepsets == sks[0].sepsets
        preq = _sum(psk.stats, "tests_required")
        out["plain_form"] = {"value": preq / pel, "unit": "CI tests/s", "ms_per_step": pel * 1e3,
                             "same_skeleton_and_sepsets": bool(same)}
        out["speedup_vs_plain"] = out["value"] / out["plain_form"]["value"]

    if not a.no_precision:
        out["precision_fp32_vs_fp64"] = precision_report(bns, handles[0], dss[0])
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(dss)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
