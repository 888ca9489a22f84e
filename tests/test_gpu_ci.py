"""GPU parity of bns_ci_batch against the oracle (Section III-B).

Counts are compared bit for bit, df exactly, G^2 within 1e-9 (FP64) or 1e-4
(FP32) relative to max(G^2, 1), p-values and decisions against the oracle's.
Sizes span several 16-sample groups and workgroup strides with ragged tails,
single-pass and multi-pass (z-chunked) tables, and degenerate inputs.
"""

import numpy as np
import pytest

from bnsynth import make_dataset

pytestmark = pytest.mark.gpu

G2_TOL = {0: 1e-4, 1: 1e-9}   # by precision: FP32_RECHECK, FP64


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


def _check(bns, orc, ds, tests, prec, alpha=0.05, lds_bytes=0, band=1e-3):
    print(f"ci_batch n={ds.n_vars} m={ds.n_samples} tests={len(tests)} prec={prec} lds={lds_bytes}",
          flush=True)
    h = bns.bns_dataset_create(ds.data, ds.cards)
    o = bns.bns_options_default(precision=prec, lds_bytes=lds_bytes, recheck_band=band)
    r = bns.bns_ci_batch(h, tests, alpha, o, want_tables=True, cards=ds.cards)
    worst = 0.0
    for t, (x, y, z) in enumerate(tests):
        g2, df, p, counts = orc.ci_test(ds.data, ds.cards, x, y, z, return_counts=True)
        assert np.array_equal(r["tables"][t].astype(np.int64), counts), f"test {t} counts"
        assert int(r["df"][t]) == df, f"test {t} df"
        err = abs(r["g2"][t] - g2) / max(abs(g2), 1.0)
        tol = G2_TOL[prec] if not (r["flags"][t] & bns.BNS_CI_RECHECKED) else 1e-9
        assert err <= tol, f"test {t}: G2 {r['g2'][t]} vs {g2} (rel {err})"
        worst = max(worst, err)
        if prec == 1 or (r["flags"][t] & bns.BNS_CI_RECHECKED):
            assert abs(r["p"][t] - p) <= 1e-9 * max(p, 1e-300) + 1e-15, f"test {t} p"
        if abs(p - alpha) > 1e-9:
            assert bool(r["flags"][t] & bns.BNS_CI_INDEPENDENT) == (p > alpha), f"test {t} decision"
    return worst


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("m", [1, 15, 16, 17, 255, 4099, 4096 * 3 + 7, 50_000])
def test_ci_batch_matches_oracle(bns, orc, prec, m):
    ds = make_dataset(12, 16, 3, 2, 5, 0.5, m, seed=1000 + m)
    rng = np.random.default_rng(m)
    _check(bns, orc, ds, _tests(rng, ds.n_vars, 60, 4), prec)


@pytest.mark.parametrize("prec", [0, 1])
def test_multi_pass_tables(bns, orc, prec):
    """Tables larger than the LDS budget are counted in z-range passes."""
    ds = make_dataset(10, 12, 3, 4, 5, 0.5, 20_000, seed=77)
    rng = np.random.default_rng(5)
    tests = _tests(rng, ds.n_vars, 20, 5)
    tests += [(0, 1, (2, 3, 4, 5, 6)), (3, 9, (0, 1, 2, 4, 5, 6, 7))]
    _check(bns, orc, ds, tests, prec, lds_bytes=8192)


def test_recheck_band_one_forces_fp64(bns, orc):
    ds = make_dataset(10, 12, 3, 2, 4, 0.5, 30_000, seed=91)
    rng = np.random.default_rng(8)
    tests = _tests(rng, ds.n_vars, 40, 3)
    h = bns.bns_dataset_create(ds.data, ds.cards)
    r32 = bns.bns_ci_batch(h, tests, 0.05, bns.bns_options_default(precision=0, recheck_band=1.0))
    r64 = bns.bns_ci_batch(h, tests, 0.05, bns.bns_options_default(precision=1))
    assert np.all(r32["flags"] & bns.BNS_CI_RECHECKED)
    assert np.array_equal(r32["g2"], r64["g2"])
    assert np.array_equal(r32["p"], r64["p"])


def test_fp32_error_is_small(bns, orc):
    """FP32 G^2 against the FP64 oracle on large-m tests (error report)."""
    ds = make_dataset(14, 20, 3, 2, 5, 0.5, 200_000, seed=123)
    rng = np.random.default_rng(9)
    worst = _check(bns, orc, ds, _tests(rng, ds.n_vars, 80, 3), 0, band=0.0)
    print("max relative FP32 G2 error", worst)
    assert worst < 1e-5


def test_degenerate_inputs(bns, orc):
    rng = np.random.default_rng(3)
    m = 5000
    data = rng.integers(0, 3, size=(5, m)).astype(np.uint8)
    data[3] = 0                      # constant column with card 1
    data[4] = data[0]                # exact copy of variable 0
    cards = np.array([3, 3, 3, 1, 3], dtype=np.uint8)

    class DS:
        pass
    ds = DS()
    ds.data, ds.cards, ds.n_vars, ds.n_samples = data, cards, 5, m
    tests = [(0, 3, ()), (3, 1, (0,)), (0, 4, ()), (0, 4, (1, 2)), (1, 2, (3,)), (0, 1, (3, 4))]
    for prec in (0, 1):
        _check(bns, orc, ds, tests, prec)
    h = bns.bns_dataset_create(data, cards)
    r = bns.bns_ci_batch(h, [(0, 3, ())], 0.05)
    assert r["df"][0] == 0 and r["p"][0] == 1.0 and r["flags"][0] & 1


def test_invalid_tests_rejected(bns):
    ds = make_dataset(6, 6, 2, 2, 3, 1.0, 100, seed=4)
    h = bns.bns_dataset_create(ds.data, ds.cards)
    for bad in [(0, 0, ()), (0, 6, ()), (0, 1, (1,)), (0, 1, (9,))]:
        with pytest.raises(bns.BnsError):
            bns.bns_ci_batch(h, [bad], 0.05)
