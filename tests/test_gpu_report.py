"""GPU tests of the verification mode, the sepset accessor and the workspace
limit of the C ABI.

- report_errors: every executed test of a search is also evaluated in FP64;
  the per-depth report covers exactly the executed tests, its FP32 errors stay
  within the FP32 tolerance (1e-4 relative to max(G^2, 1)), and the search's
  results are those of the oracle (the report does not change decisions).
- bns_skeleton_sepset answers every pair, in either order, as the oracle's
  sepsets say (Algorithm 1: the first accepting set; kept edges report -1).
- workspace_mb: a limit below what a call needs gives BNS_E_NOMEM before any
  device work, a sufficient one runs normally.
"""

import ctypes

import numpy as np
import pytest

from bnsynth import make_config
from golden_util import compare_skeleton, expand, load_golden

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bns():
    import paper_2212_04259_amd as b
    b.load()
    return b


@pytest.mark.parametrize("k", [1, 2, 3])
def test_report_errors_covers_every_executed_test(bns, k):
    g = load_golden(k)["datasets"][0]
    ds = make_config(k)[0]
    print(f"report_errors cfg{k}", flush=True)
    o = bns.bns_options_default(report_errors=1)
    got = bns.bns_pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth, o)
    compare_skeleton(got, g, f"cfg{k} report_errors")
    for s in got.stats:
        assert s["err_tests"] == s["tests_executed"], s
        assert 0.0 <= s["err_p50"] <= s["err_p99"] <= s["err_max"] < 1e-4, s
        # the FP32-only decision never differs from FP64 outside the
        # re-check band; a flip would have been re-checked
        assert s["err_flips"] <= s["rechecks"], s


def test_report_errors_split_and_multipass(bns):
    # split depths (merged tables re-read for FP64) and z-range passes
    # (counted again for FP64) in verification mode
    g = load_golden(2)["datasets"][0]
    ds = make_config(2)[0]
    for opts in (dict(split_min_samples=1024, units_per_group=16), dict(lds_bytes=8192)):
        print(f"report_errors cfg2 {opts}", flush=True)
        o = bns.bns_options_default(report_errors=1, **opts)
        got = bns.bns_pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth, o)
        compare_skeleton(got, g, f"cfg2 report_errors {opts}")
        assert all(s["err_tests"] == s["tests_executed"] for s in got.stats)
        assert max(s["err_max"] for s in got.stats) < 1e-4


def test_report_errors_off_and_fp64(bns):
    ds = make_config(1)[0]
    for o in (bns.bns_options_default(), bns.bns_options_default(report_errors=1, precision=1)):
        got = bns.bns_pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth, o)
        assert all(s["err_tests"] == 0 and s["err_max"] == 0.0 for s in got.stats)


def test_sepset_accessor_every_pair(bns):
    g = load_golden(2)["datasets"][0]
    ds = make_config(2)[0]
    adj, depth, sep = expand(g)
    L = bns.load()
    o = bns.bns_options_default()
    h = ctypes.c_void_p()
    print("sepset accessor cfg2", flush=True)
    st = L.bns_pc_skeleton(ds.data.ctypes.data_as(ctypes.c_void_p), ds.n_samples, ds.n_vars,
                           ds.cards.ctypes.data_as(ctypes.c_void_p), ds.alpha, ds.max_depth,
                           ctypes.byref(o), ctypes.byref(h))
    assert st == 0, L.bns_last_error()
    try:
        n = ds.n_vars
        buf = (ctypes.c_int32 * 32)()
        ln, rd = ctypes.c_int32(), ctypes.c_int32()
        for i in range(n):
            for j in range(n):
                if i == j:
                    assert L.bns_skeleton_sepset(h, i, j, buf, 32, ctypes.byref(ln), ctypes.byref(rd)) == 1
                    continue
                assert L.bns_skeleton_sepset(h, i, j, buf, 32, ctypes.byref(ln), ctypes.byref(rd)) == 0
                a, b = min(i, j), max(i, j)
                if adj[a, b]:
                    assert ln.value == -1 and rd.value == -1, (i, j)
                else:
                    assert ln.value == depth[a, b] == rd.value, (i, j)
                    assert tuple(buf[:ln.value]) == sep[(a, b)], (i, j)
        # a short buffer receives the first members, the length is complete
        deep = [(a, b) for (a, b), S in sep.items() if len(S) >= 2]
        a, b = deep[0]
        assert L.bns_skeleton_sepset(h, a, b, buf, 1, ctypes.byref(ln), None) == 0
        assert ln.value == len(sep[(a, b)]) and buf[0] == sep[(a, b)][0]
        # out-of-range pairs are rejected
        for bad in ((-1, 0), (0, n), (n, 0)):
            assert L.bns_skeleton_sepset(h, bad[0], bad[1], buf, 32, ctypes.byref(ln), None) == 1
    finally:
        L.bns_skeleton_free(h)


def test_workspace_limit(bns):
    ds = make_config(2)[0]
    h = bns.bns_dataset_create(ds.data, ds.cards)
    print("workspace limit cfg2", flush=True)
    with pytest.raises(bns.BnsError) as ei:
        bns.bns_pc_skeleton_dataset(h, ds.alpha, ds.max_depth, bns.bns_options_default(workspace_mb=1))
    assert ei.value.status == 4 and "workspace" in str(ei.value)
    # the split-merge tables alone take 32 MiB; 256 MiB is enough for the 60-variable workload
    got = bns.bns_pc_skeleton_dataset(h, ds.alpha, ds.max_depth, bns.bns_options_default(workspace_mb=256))
    compare_skeleton(got, load_golden(2)["datasets"][0], "cfg2 workspace 256 MiB")
    tests = [(0, 1, ())] * 100_000
    with pytest.raises(bns.BnsError) as ei:
        bns.bns_ci_batch(h, tests, ds.alpha, bns.bns_options_default(workspace_mb=1))
    assert ei.value.status == 4
    r = bns.bns_ci_batch(h, tests[:10], ds.alpha, bns.bns_options_default(workspace_mb=1))
    assert np.all(r["g2"] == r["g2"][0])
