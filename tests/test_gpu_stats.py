"""GPU parity of the other CI statistics on the same counting kernels: Pearson
X^2 (Section II) and the adjusted degrees of freedom (the variant of reading
R1), against the oracle run live.

bns_ci_batch: counts bit-exact, df exact, the statistic within 1e-4 (FP32) or
1e-9 (FP64) of max(stat, 1), decisions equal away from knife edges.  Skeleton
searches (batched FP32 + re-check and FP64, plain form): skeleton, removal
depths, sepsets and per-depth test counts identical to the oracle's with the
same statistic and df rule.
"""

import numpy as np
import pytest

from bnsynth import make_config, make_dataset
from golden_util import compare_with_oracle

pytestmark = pytest.mark.gpu

TOL = {0: 1e-4, 1: 1e-9}


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


@pytest.mark.parametrize("stat,df_rule", [(1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("m", [37, 4099, 60_000])
def test_ci_batch_statistics_match_oracle(bns, orc, stat, df_rule, prec, m):
    ds = make_dataset(12, 16, 3, 2, 5, 0.5, m, seed=5000 + m)
    rng = np.random.default_rng(m + 17)
    tests = _tests(rng, ds.n_vars, 60, 4)
    print(f"ci_batch stat={stat} df_rule={df_rule} prec={prec} m={m}", flush=True)
    h = bns.bns_dataset_create(ds.data, ds.cards)
    o = bns.bns_options_default(precision=prec, statistic=stat, df_rule=df_rule)
    r = bns.bns_ci_batch(h, tests, 0.05, o, want_tables=True, cards=ds.cards)
    for t, (x, y, z) in enumerate(tests):
        s, df, p, counts = orc.ci_test(ds.data, ds.cards, x, y, z, return_counts=True, statistic=stat,
                                       df_rule=df_rule)
        assert np.array_equal(r["tables"][t].astype(np.int64), counts), f"test {t} counts"
        assert int(r["df"][t]) == df, f"test {t} df {r['df'][t]} vs {df}"
        tol = TOL[prec] if not (r["flags"][t] & bns.BNS_CI_RECHECKED) else 1e-9
        assert abs(r["g2"][t] - s) <= tol * max(abs(s), 1.0), f"test {t}: {r['g2'][t]} vs {s}"
        if abs(p - 0.05) > 1e-9:
            assert bool(r["flags"][t] & 1) == (p > 0.05), f"test {t} decision"


def test_multi_pass_tables_adjusted_x2(bns, orc):
    # z-range passes: the adjusted df and X^2 summed over passes
    ds = make_dataset(10, 12, 3, 4, 5, 0.5, 3_000, seed=78)
    tests = [(0, 1, (2, 3, 4, 5, 6)), (3, 9, (0, 1, 2, 4, 5, 6)), (1, 2, (0, 3, 4, 5))]
    h = bns.bns_dataset_create(ds.data, ds.cards)
    for prec in (0, 1):
        o = bns.bns_options_default(precision=prec, statistic=1, df_rule=1, lds_bytes=8192)
        r = bns.bns_ci_batch(h, tests, 0.05, o)
        for t, (x, y, z) in enumerate(tests):
            s, df, p = orc.ci_test(ds.data, ds.cards, x, y, z, statistic=1, df_rule=1)
            assert int(r["df"][t]) == df
            assert abs(r["g2"][t] - s) <= TOL[prec] * max(s, 1.0)


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("stat,df_rule", [(1, 0), (0, 1), (1, 1)])
def test_skeleton_statistics_match_oracle(bns, orc, k, stat, df_rule):
    ds = make_config(k)[0]
    ref = orc.pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth, statistic=stat, df_rule=df_rule)
    assert ref.knife_edges == 0
    forms = [dict(), dict(precision=1)] + ([dict(form=1, precision=1)] if k == 1 else [])
    for extra in forms:
        print(f"skeleton cfg{k} stat={stat} df_rule={df_rule} {extra}", flush=True)
        o = bns.bns_options_default(statistic=stat, df_rule=df_rule, **extra)
        got = bns.bns_pc_skeleton(ds.data, ds.cards, ds.alpha, ds.max_depth, o)
        compare_with_oracle(got, ref, f"cfg{k} stat={stat} df_rule={df_rule} {extra}")


@pytest.mark.parametrize("seed", range(4))
def test_sparse_tables_adjusted_df_skeleton(bns, orc, seed):
    # few samples over many cells: empty categories and strata everywhere
    rng = np.random.default_rng(seed)
    n = int(rng.integers(6, 14))
    ds = make_dataset(n, int(1.3 * n), 3, 3, 5, 0.5, int(rng.integers(30, 400)), seed=880 + seed)
    for stat in (0, 1):
        ref = orc.pc_skeleton(ds.data, ds.cards, 0.05, -1, statistic=stat, df_rule=1)
        if ref.knife_edges:
            continue
        for form in (0, 1):
            o = bns.bns_options_default(statistic=stat, df_rule=1, form=form)
            got = bns.bns_pc_skeleton(ds.data, ds.cards, 0.05, -1, o)
            compare_with_oracle(got, ref, f"sparse seed {seed} stat {stat} form {form}")
