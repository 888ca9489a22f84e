"""GPU test of bns_ci_batch_noalloc, the allocation-free variant of
bns_ci_batch: called through the C ABI twice in a row (the second call
smaller, so stale scratch contents from the first would show), its results
must equal bns_ci_batch's on the same tests bit for bit (the same kernels),
and match the oracle's counts-derived G^2, df and decisions to the FP32
tolerance; a call beyond the fixed scratch size fails with BNS_E_NOMEM."""

import ctypes

import numpy as np
import pytest

from bnsynth import make_dataset

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bns():
    import paper_2212_04259_amd as b
    b.load()
    return b


def _tests(rng, n, count, dmax):
    out = []
    for _ in range(count):
        d = int(rng.integers(0, dmax + 1))
        vs = rng.permutation(n)[: d + 2]
        out.append((int(vs[0]), int(vs[1]), tuple(int(v) for v in vs[2:])))
    return out


def _raw_noalloc(bns, h, tests, alpha):
    # the entry point called directly through the C ABI
    L = bns.load()
    n = len(tests)
    from paper_2212_04259_amd._lib import bns_ci_test
    arr = (bns_ci_test * n)()
    zs = []
    for t, (x, y, z) in enumerate(tests):
        arr[t].x, arr[t].y, arr[t].n_z, arr[t].z_offset = x, y, len(z), len(zs)
        zs.extend(z)
    zp = np.asarray(zs or [0], dtype=np.int32)
    g2 = np.zeros(n)
    df = np.zeros(n, dtype=np.int64)
    p = np.zeros(n)
    fl = np.zeros(n, dtype=np.int32)
    o = bns.bns_options_default()
    vp = ctypes.c_void_p
    st = L.bns_ci_batch_noalloc(h.handle, ctypes.cast(arr, vp), n, zp.ctypes.data_as(vp), len(zs), alpha,
                                ctypes.byref(o), g2.ctypes.data_as(vp), df.ctypes.data_as(vp),
                                p.ctypes.data_as(vp), fl.ctypes.data_as(vp))
    assert st == 0, L.bns_last_error()
    return dict(g2=g2, df=df, p=p, flags=fl)


def test_noalloc_matches_ci_batch_twice(bns, orc):
    ds = make_dataset(14, 18, 3, 2, 5, 0.5, 30_011, seed=2718)
    h = bns.bns_dataset_create(ds.data, ds.cards)
    rng = np.random.default_rng(11)
    big = _tests(rng, ds.n_vars, 3000, 4)
    small = _tests(rng, ds.n_vars, 37, 3)
    for label, tests in (("first call, 3000 tests", big), ("second call, 37 tests", small)):
        print(f"noalloc {label}", flush=True)
        got = _raw_noalloc(bns, h, tests, ds.alpha)
        ref = bns.bns_ci_batch(h, tests, ds.alpha)
        for k in ("g2", "df", "p", "flags"):
            assert np.array_equal(got[k], ref[k]), (label, k)
        for t in range(0, len(tests), max(1, len(tests) // 40)):
            x, y, z = tests[t]
            g2, df, p = orc.ci_test(ds.data, ds.cards, x, y, z)
            assert got["df"][t] == df
            assert abs(got["g2"][t] - g2) <= 1e-4 * max(abs(g2), 1.0)
            if abs(p - ds.alpha) > 1e-9:
                assert bool(got["flags"][t] & 1) == (p > ds.alpha)


def test_noalloc_rejects_oversized_calls(bns):
    ds = make_dataset(6, 6, 2, 2, 3, 1.0, 1000, seed=5)
    h = bns.bns_dataset_create(ds.data, ds.cards)
    too_many = bns.NOALLOC_SCRATCH_BYTES // 44 + 1000
    print(f"noalloc oversized call ({too_many} tests)", flush=True)
    with pytest.raises(bns.BnsError) as ei:
        bns.bns_ci_batch_noalloc(h, [(0, 1, ())] * too_many, 0.05)
    assert ei.value.status == 4 and "scratch" in str(ei.value)
    # the entry point still works after a rejected call
    r = bns.bns_ci_batch_noalloc(h, [(0, 1, ()), (2, 3, (4,))], 0.05)
    ref = bns.bns_ci_batch(h, [(0, 1, ()), (2, 3, (4,))], 0.05)
    assert np.array_equal(r["g2"], ref["g2"]) and np.array_equal(r["flags"], ref["flags"])
