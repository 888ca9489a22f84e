"""Pins of the oracle's other CI statistics (Section II names Pearson's X^2 as
an alternative test on the same contingency table; the adjusted degrees of
freedom are the variant of reading R1 that drops empty categories and strata).

Nothing re-types the oracle's formulas: X^2 is checked against scipy's Pearson
statistic (chi2_contingency without continuity correction) on 2-D tables and
strata, against the closed form m (ad - bc)^2 / ((a+b)(c+d)(a+c)(b+d)) of a
2x2 table, and against invariances; the adjusted df against scipy's dof of
each stratum's table with its empty rows and columns removed, counted by
brute force from the data.
"""

import numpy as np
import pytest
from scipy.stats import chi2, chi2_contingency

from test_oracle_ci import _brute_counts, _data_from_table, _rand_data


def _stratum_tables(data, cards, x, y, z):
    """2-D tables of every stratum (in zc order) from brute-force counts."""
    counts = _brute_counts(data, cards, x, y, z)
    rx, ry = int(cards[x]), int(cards[y])
    zr = [range(int(cards[v])) for v in z]
    import itertools
    out = []
    for zs in itertools.product(*reversed(zr)) if z else [()]:
        zs = tuple(reversed(zs))
        t = np.zeros((rx, ry), dtype=np.int64)
        for xv in range(rx):
            for yv in range(ry):
                t[xv, yv] = counts[(xv, yv) + zs]
        out.append(t)
    return out


def _scipy_x2(t):
    t = t[t.sum(1) > 0][:, t.sum(0) > 0]
    if t.size == 0 or t.shape[0] < 2 or t.shape[1] < 2:
        return 0.0
    return float(chi2_contingency(t, correction=False)[0])


def _scipy_dof(t):
    t = t[t.sum(1) > 0][:, t.sum(0) > 0]
    if t.sum() == 0:
        return 0
    return (t.shape[0] - 1) * (t.shape[1] - 1)


@pytest.mark.parametrize("seed", range(10))
def test_x2_matches_scipy_per_stratum(orc, seed):
    rng = np.random.default_rng(300 + seed)
    data, cards = _rand_data(rng, 6, int(rng.integers(40, 3000)), 2, 4)
    x, y = 0, 1
    z = tuple(int(v) for v in rng.choice(np.arange(2, 6), size=int(rng.integers(0, 3)), replace=False))
    x2, df, p = orc.ci_test(data, cards, x, y, z, statistic=orc.STAT_X2)
    tabs = _stratum_tables(data, cards, x, y, z)
    want = sum(_scipy_x2(t) for t in tabs)
    assert x2 == pytest.approx(want, rel=1e-11, abs=1e-11)
    assert df == (int(cards[x]) - 1) * (int(cards[y]) - 1) * int(np.prod([int(cards[v]) for v in z]))
    assert p == pytest.approx(chi2.sf(x2, df), rel=1e-10, abs=1e-300)


def test_x2_closed_form_2x2(orc):
    for a, b, c, d in [(30, 10, 20, 40), (5, 15, 25, 5), (1, 0, 0, 1), (7, 3, 2, 9)]:
        data, cards = _data_from_table(np.array([[[a, b], [c, d]]]).transpose(1, 2, 0))
        x2, df, _ = orc.ci_test(data, cards, 0, 1, (), statistic=orc.STAT_X2)
        m = a + b + c + d
        # table rows are x, columns y: N[x=0,y=0]=a, N[x=0,y=1]=b, N[x=1,y=0]=c, N[x=1,y=1]=d
        want = m * (a * d - b * c) ** 2 / ((a + b) * (c + d) * (a + c) * (b + d))
        assert x2 == pytest.approx(want, rel=1e-13)
        assert df == 1


@pytest.mark.parametrize("seed", range(5))
def test_x2_invariances(orc, seed):
    rng = np.random.default_rng(700 + seed)
    data, cards = _rand_data(rng, 5, 2000, 2, 4)
    base = orc.ci_test(data, cards, 0, 1, (2, 3), statistic=1)[0]
    assert base >= 0.0
    # X <-> Y
    assert orc.ci_test(data, cards, 1, 0, (2, 3), statistic=1)[0] == pytest.approx(base, rel=1e-12)
    # order of Z
    assert orc.ci_test(data, cards, 0, 1, (3, 2), statistic=1)[0] == pytest.approx(base, rel=1e-12)
    # relabelled categories of X
    d2 = data.copy()
    perm = rng.permutation(int(cards[0]))
    d2[0] = perm[data[0]]
    assert orc.ci_test(d2, cards, 0, 1, (2, 3), statistic=1)[0] == pytest.approx(base, rel=1e-12)
    # an exact product table gives 0
    t = np.outer([2, 4, 6], [3, 1]).reshape(3, 2, 1)
    dp, cp = _data_from_table(t)
    assert orc.ci_test(dp, cp, 0, 1, (), statistic=1)[0] == pytest.approx(0.0, abs=1e-12)


@pytest.mark.parametrize("seed", range(10))
def test_adjusted_df_matches_reduced_tables(orc, seed):
    rng = np.random.default_rng(900 + seed)
    # few samples over many cells: empty rows, columns and strata are common
    data, cards = _rand_data(rng, 6, int(rng.integers(5, 60)), 2, 5)
    z = (2, 3, 4)[: int(rng.integers(0, 4))]
    for stat in (orc.STAT_G2, orc.STAT_X2):
        s_adj, df_adj, p_adj = orc.ci_test(data, cards, 0, 1, z, statistic=stat, df_rule=orc.DF_ADJUSTED)
        s_dec, df_dec, _ = orc.ci_test(data, cards, 0, 1, z, statistic=stat)
        assert s_adj == s_dec  # the rule changes df only
        want = sum(_scipy_dof(t) for t in _stratum_tables(data, cards, 0, 1, z))
        assert df_adj == want
        assert df_adj <= df_dec
        if df_adj == 0:
            assert p_adj == 1.0
        else:
            assert p_adj == pytest.approx(chi2.sf(s_adj, df_adj), rel=1e-10, abs=1e-300)


def test_adjusted_df_full_tables_equal_declared(orc):
    rng = np.random.default_rng(5)
    data, cards = _rand_data(rng, 4, 50_000, 2, 3)
    for z in ((), (2,), (2, 3)):
        a = orc.ci_test(data, cards, 0, 1, z, df_rule=orc.DF_ADJUSTED)
        d = orc.ci_test(data, cards, 0, 1, z)
        assert a == d


def test_adjusted_df_planted_empty_categories(orc):
    # x has 4 declared categories but uses 2; y uses all 3: df = (2-1)(3-1) = 2
    t = np.zeros((4, 3, 1), dtype=np.int64)
    t[0] = [[5], [3], [7]]
    t[2] = [[2], [9], [4]]
    data, cards = _data_from_table(t)
    s, df, p = orc.ci_test(data, cards, 0, 1, (), statistic=1, df_rule=1)
    assert df == 2
    assert orc.ci_test(data, cards, 0, 1, ())[1] == 6
    # a single non-empty row: df 0, p 1 (independent)
    t1 = np.zeros((3, 3, 1), dtype=np.int64)
    t1[1] = [[4], [5], [6]]
    d1, c1 = _data_from_table(t1)
    s, df, p = orc.ci_test(d1, c1, 0, 1, (), df_rule=1)
    assert df == 0 and p == 1.0


def test_pc_skeleton_with_other_statistics_runs_the_same_order(orc):
    # The driver is unchanged: with X^2 the tests are the same sequence of
    # (x, y, S) as long as the decisions agree; on a strongly dependent chain
    # both statistics recover the same skeleton.
    from bnsynth import forward_sample
    rng = np.random.default_rng(3)
    cards = np.array([3, 3, 3, 3], dtype=np.uint8)
    edges = [(0, 1), (1, 2), (2, 3)]
    cpts = {}
    for v in range(4):
        parents = [a for a, b in edges if b == v]
        rows = 3 ** len(parents)
        cp = np.full((rows, 3), 0.05)
        for r in range(rows):
            cp[r, r % 3] = 0.9
        cpts[v] = cp / cp.sum(1, keepdims=True)
    parents = [[a for a, b in edges if b == v] for v in range(4)]
    data = forward_sample(rng, [0, 1, 2, 3], parents, cards, cpts, 20_000)
    r_g2 = orc.pc_skeleton(data, cards, 0.01)
    r_x2 = orc.pc_skeleton(data, cards, 0.01, statistic=1)
    r_adj = orc.pc_skeleton(data, cards, 0.01, statistic=1, df_rule=1)
    truth = np.zeros((4, 4), dtype=np.uint8)
    for a, b in edges:
        truth[a, b] = truth[b, a] = 1
    for r in (r_g2, r_x2, r_adj):
        assert np.array_equal(r.adj, truth)
