"""Pins of the oracle's CI test (Section III-B): counts, marginals, G^2, df.

Nothing here re-types the oracle's formulas: counts are checked by direct
comparison of rows, G^2 by a 50-digit mpmath evaluation of the definition from
brute-force counts, and by scipy's log-likelihood contingency statistic,
information-theoretic identities and invariances.
"""

import itertools
import math

import mpmath
import numpy as np
import pytest
from scipy.stats import chi2_contingency

mpmath.mp.dps = 50


def _rand_data(rng, n, m, lo=2, hi=4):
    cards = rng.integers(lo, hi + 1, n).astype(np.uint8)
    data = np.stack([rng.integers(0, int(c), m) for c in cards]).astype(np.uint8)
    return data, cards


def _brute_counts(data, cards, x, y, z):
    """N[(xv, yv, zvals)] by comparing every row against every cell."""
    out = {}
    ranges = [range(int(cards[x])), range(int(cards[y]))] + [range(int(cards[v])) for v in z]
    for cell in itertools.product(*ranges):
        mask = (data[x] == cell[0]) & (data[y] == cell[1])
        for k, v in enumerate(z):
            mask &= data[v] == cell[2 + k]
        out[cell] = int(mask.sum())
    return out


def _cell_index(cell, cards, x, y, z):
    xv, yv, zs = cell[0], cell[1], cell[2:]
    zc, mult = 0, 1
    for k, v in enumerate(z):
        zc += zs[k] * mult
        mult *= int(cards[v])
    return xv + int(cards[x]) * (yv + int(cards[y]) * zc)


def _mp_g2(counts, cards, x, y, z):
    """G^2 = 2 sum N ln(N N_++z / (N_x+z N_+yz)) with exact integer marginals."""
    nxz, nyz, nz = {}, {}, {}
    for (xv, yv, *zs), c in counts.items():
        zs = tuple(zs)
        nxz[(xv, zs)] = nxz.get((xv, zs), 0) + c
        nyz[(yv, zs)] = nyz.get((yv, zs), 0) + c
        nz[zs] = nz.get(zs, 0) + c
    s = mpmath.mpf(0)
    for (xv, yv, *zs), c in counts.items():
        if c == 0:
            continue
        zs = tuple(zs)
        s += c * mpmath.log(mpmath.mpf(c * nz[zs]) / (nxz[(xv, zs)] * nyz[(yv, zs)]))
    return 2 * s


def _data_from_table(table3):
    """Rows realising a table N[x][y][z] (z is one conditioning variable)."""
    t = np.asarray(table3, dtype=np.int64)
    if t.ndim == 2:
        t = t[:, :, None]
    rx, ry, rz = t.shape
    cols = [[], [], []]
    for xv in range(rx):
        for yv in range(ry):
            for zv in range(rz):
                c = int(t[xv, yv, zv])
                cols[0] += [xv] * c
                cols[1] += [yv] * c
                cols[2] += [zv] * c
    data = np.array(cols, dtype=np.uint8)
    cards = np.array([rx, ry, rz], dtype=np.uint8)
    return data, cards


@pytest.mark.parametrize("seed", range(12))
def test_counts_match_brute_force(orc, seed):
    rng = np.random.default_rng(seed)
    n, m = 6, int(rng.integers(1, 65))
    data, cards = _rand_data(rng, n, m, 2, 4)
    d = int(rng.integers(0, 4))
    vs = rng.permutation(n)[: d + 2]
    x, y, z = int(vs[0]), int(vs[1]), [int(v) for v in vs[2:]]
    _, _, _, got = orc.ci_test(data, cards, x, y, z, return_counts=True)
    brute = _brute_counts(data, cards, x, y, z)
    assert got.sum() == m
    assert len(got) == len(brute)
    for cell, c in brute.items():
        assert got[_cell_index(cell, cards, x, y, z)] == c
    # Cross-check with numpy's multi-dimensional histogram.
    sample = np.stack([data[v] for v in [x, y] + z], axis=1)
    bins = [np.arange(int(cards[v]) + 1) - 0.5 for v in [x, y] + z]
    h, _ = np.histogramdd(sample, bins=bins)
    for cell, c in brute.items():
        assert int(h[cell]) == c


@pytest.mark.parametrize("seed", range(12))
def test_g2_matches_mpmath_definition(orc, seed):
    rng = np.random.default_rng(100 + seed)
    n, m = 6, int(rng.integers(20, 400))
    data, cards = _rand_data(rng, n, m, 2, 4)
    d = int(rng.integers(0, 3))
    vs = rng.permutation(n)[: d + 2]
    x, y, z = int(vs[0]), int(vs[1]), [int(v) for v in vs[2:]]
    g2, df, p = orc.ci_test(data, cards, x, y, z)
    ref = _mp_g2(_brute_counts(data, cards, x, y, z), cards, x, y, z)
    assert abs(g2 - float(ref)) <= 1e-12 * max(1.0, abs(float(ref)))
    assert df == (int(cards[x]) - 1) * (int(cards[y]) - 1) * int(np.prod([int(cards[v]) for v in z]))
    assert g2 >= 0.0
    assert 0.0 <= p <= 1.0


def test_fixed_tables_against_mpmath_and_closed_forms(orc):
    # 2x2 table: df 1, p = erfc(sqrt(G2/2)).
    data, cards = _data_from_table([[30, 10], [20, 40]])
    g2, df, p = orc.ci_test(data, cards, 0, 1)
    ref = _mp_g2(_brute_counts(data, cards, 0, 1, []), cards, 0, 1, [])
    assert df == 1
    assert abs(g2 - float(ref)) < 1e-12 * float(ref)
    assert abs(float(ref) - 17.260924347106855646) < 1e-15
    assert abs(p - float(mpmath.erfc(mpmath.sqrt(ref / 2)))) < 1e-12 * p
    # Two strata conditioning on z: df 2, p = exp(-G2/2).
    data, cards = _data_from_table(np.stack([[[30, 10], [20, 40]], [[5, 15], [25, 5]]], axis=2))
    g2, df, p = orc.ci_test(data, cards, 0, 1, [2])
    ref = _mp_g2(_brute_counts(data, cards, 0, 1, [2]), cards, 0, 1, [2])
    assert df == 2
    assert abs(g2 - float(ref)) < 1e-12 * float(ref)
    assert abs(p - float(mpmath.exp(-ref / 2))) < 1e-12 * p
    # 3x3 with a zero cell: df 4.
    data, cards = _data_from_table([[12, 0, 7], [3, 9, 4], [6, 5, 10]])
    g2, df, p = orc.ci_test(data, cards, 0, 1)
    ref = _mp_g2(_brute_counts(data, cards, 0, 1, []), cards, 0, 1, [])
    assert df == 4
    assert abs(g2 - float(ref)) < 1e-12 * float(ref)
    # even df: Poisson tail exp(-x) sum_{k<df/2} x^k/k!
    x = ref / 2
    tail = mpmath.exp(-x) * sum(x ** k / mpmath.factorial(k) for k in range(2))
    assert abs(p - float(tail)) < 1e-12 * p
    # A product table has G^2 = 0 exactly and p = 1.
    data, cards = _data_from_table([[2, 4], [3, 6]])
    g2, df, p = orc.ci_test(data, cards, 0, 1)
    assert g2 == 0.0 and p == 1.0


@pytest.mark.parametrize("seed", range(8))
def test_g2_equals_scipy_log_likelihood(orc, seed):
    rng = np.random.default_rng(200 + seed)
    rx, ry = int(rng.integers(2, 6)), int(rng.integers(2, 6))
    table = rng.integers(1, 60, size=(rx, ry))
    data, cards = _data_from_table(table)
    g2, df, p = orc.ci_test(data, cards, 0, 1)
    stat, pval, dof, _ = chi2_contingency(table, correction=False, lambda_="log-likelihood")
    assert dof == df
    assert abs(g2 - stat) <= 1e-10 * max(1.0, stat)
    assert abs(p - pval) <= 1e-10 * max(pval, 1e-300) + 1e-300


@pytest.mark.parametrize("seed", range(6))
def test_g2_invariances(orc, seed):
    rng = np.random.default_rng(300 + seed)
    n, m = 5, 500
    data, cards = _rand_data(rng, n, m, 2, 4)
    # make y depend on x so that G^2 is not tiny
    data[1] = (data[0] + (rng.random(m) < 0.3)) % cards[1]
    x, y, z = 0, 1, [2, 3]
    g2, df, _ = orc.ci_test(data, cards, x, y, z)
    # X <-> Y symmetry
    g2b, dfb, _ = orc.ci_test(data, cards, y, x, z)
    assert abs(g2 - g2b) <= 1e-12 * g2 and df == dfb
    # permuting the order of Z
    g2c, _, _ = orc.ci_test(data, cards, x, y, z[::-1])
    assert abs(g2 - g2c) <= 1e-12 * g2
    # relabelling categories of x, y and a z variable
    d2 = data.copy()
    for v in (0, 1, 2):
        perm = rng.permutation(int(cards[v]))
        d2[v] = perm[data[v]]
    g2d, _, _ = orc.ci_test(d2, cards, x, y, z)
    assert abs(g2 - g2d) <= 1e-12 * g2
    # stratum additivity: G^2(X,Y|Z) = sum over strata of the marginal G^2
    # computed on the rows of that stratum.
    total = 0.0
    for zv in itertools.product(range(int(cards[2])), range(int(cards[3]))):
        rows = (data[2] == zv[0]) & (data[3] == zv[1])
        if rows.sum() == 0:
            continue
        sub = np.ascontiguousarray(data[:, rows])
        total += orc.ci_test(sub, cards, x, y, [])[0]
    assert abs(g2 - total) <= 1e-10 * g2


@pytest.mark.parametrize("seed", range(4))
def test_g2_is_twice_m_times_conditional_mutual_information(orc, seed):
    rng = np.random.default_rng(400 + seed)
    m = 1000
    data, cards = _rand_data(rng, 4, m, 2, 3)
    data[1] = (data[0] * data[2]) % cards[1]
    g2, _, _ = orc.ci_test(data, cards, 0, 1, [2])
    # I(X;Y|Z) = H(X,Z) + H(Y,Z) - H(Z) - H(X,Y,Z) with empirical plug-in entropies.
    def H(cols):
        keys = np.zeros(m, dtype=np.int64)
        for c in cols:
            keys = keys * 256 + data[c]
        _, cnt = np.unique(keys, return_counts=True)
        pr = cnt / m
        return float(-(pr * np.log(pr)).sum())
    cmi = H([0, 2]) + H([1, 2]) - H([2]) - H([0, 1, 2])
    assert abs(g2 - 2 * m * cmi) <= 1e-8 * max(1.0, g2)


def test_card_one_variable_gives_df_zero_and_p_one(orc):
    data = np.array([[0, 1, 0, 1], [0, 0, 0, 0]], dtype=np.uint8)
    cards = np.array([2, 1], dtype=np.uint8)
    g2, df, p = orc.ci_test(data, cards, 0, 1)
    assert df == 0 and p == 1.0 and g2 == 0.0


def test_bad_arguments_rejected(orc):
    data = np.zeros((3, 10), dtype=np.uint8)
    cards = np.array([2, 2, 2], dtype=np.uint8)
    with pytest.raises(ValueError):
        orc.ci_test(data, cards, 0, 0)
    with pytest.raises(ValueError):
        orc.ci_test(data, cards, 0, 1, [1])
    with pytest.raises(ValueError):
        orc.ci_test(data, cards, 0, 5)


def test_log_is_natural(orc):
    # For a perfectly dependent 2x2 table with n rows per diagonal cell,
    # G^2 = 2 * 2n * ln 2 exactly (natural logarithm).
    data, cards = _data_from_table([[50, 0], [0, 50]])
    g2, _, _ = orc.ci_test(data, cards, 0, 1)
    assert abs(g2 - 200 * math.log(2)) < 1e-12 * g2
