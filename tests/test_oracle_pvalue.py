"""Pins of the oracle's chi-square tail Q(df/2, G^2/2) (Section III-B).

Checked against closed forms (df = 1, 2, even df), scipy's independent
``gammaincc`` and chi-square quantiles, and mpmath.
"""

import math

import mpmath
import numpy as np
import pytest
from scipy import special, stats


def test_df2_closed_form(orc):
    for g2 in [0.01, 0.5, 3.0, 5.991464547107983, 9.210340371976182, 40.0, 300.0]:
        assert abs(orc.chi2_sf(g2, 2) - math.exp(-g2 / 2)) <= 1e-14 * math.exp(-g2 / 2)


def test_df1_closed_form(orc):
    for g2 in [1e-6, 0.3, 1.0, 3.8414588206941285, 6.634896601021217, 25.0, 200.0]:
        ref = math.erfc(math.sqrt(g2 / 2))
        assert abs(orc.chi2_sf(g2, 1) - ref) <= 1e-13 * ref


@pytest.mark.parametrize("df", [4, 6, 10, 20, 64])
def test_even_df_poisson_tail(orc, df):
    for g2 in [0.5 * df, df - 1.0, 1.0 * df, 1.5 * df, 2.5 * df]:
        x = mpmath.mpf(g2) / 2
        ref = mpmath.exp(-x) * mpmath.fsum(x ** k / mpmath.factorial(k) for k in range(df // 2))
        assert abs(orc.chi2_sf(g2, df) - float(ref)) <= 1e-12 * float(ref)


def test_gammaincc_grid(orc):
    for a in [0.5, 1.0, 1.5, 2.5, 8.0, 30.5, 100.0, 512.0, 2000.0, 5000.0]:
        for f in np.linspace(0.5, 2.0, 13):
            x = a * f
            ref = special.gammaincc(a, x)
            got = orc.gamma_q(a, x)
            if ref >= 1e-10:
                assert abs(got - ref) <= 1e-11 * ref, (a, x, got, ref)
            else:
                assert abs(got - ref) <= 1e-20


@pytest.mark.parametrize("alpha", [0.05, 0.01])
@pytest.mark.parametrize("df", [1, 2, 3, 4, 9, 16, 48, 100, 1000, 10000])
def test_p_at_critical_value_is_alpha(orc, alpha, df):
    crit = stats.chi2.ppf(1 - alpha, df)
    assert abs(orc.chi2_sf(crit, df) - alpha) <= 1e-11


def test_printed_critical_values(orc):
    # Textbook chi-square critical values.
    assert abs(orc.chi2_sf(3.8414588206941285, 1) - 0.05) < 1e-12
    assert abs(orc.chi2_sf(5.991464547107983, 2) - 0.05) < 1e-12
    assert abs(orc.chi2_sf(6.634896601021217, 1) - 0.01) < 1e-12
    assert abs(orc.chi2_sf(9.210340371976182, 2) - 0.01) < 1e-12
    assert abs(orc.chi2_sf(10233.748897677937, 10000) - 0.05) < 1e-9


def test_mpmath_large_df(orc):
    mpmath.mp.dps = 40
    for a, x in [(5000.0, 5100.0), (5000.0, 4900.0), (25000.0, 25300.0), (0.5, 1e-8), (3.0, 60.0)]:
        ref = mpmath.gammainc(a, x, mpmath.inf, regularized=True)
        got = orc.gamma_q(a, x)
        assert abs(got - float(ref)) <= 1e-11 * float(ref)


def test_monotone_and_bounds(orc):
    for df in [1, 3, 12, 400]:
        xs = np.linspace(0, 4 * df + 20, 400)
        ps = [orc.chi2_sf(x, df) for x in xs]
        assert all(0.0 <= p <= 1.0 for p in ps)
        assert all(a >= b for a, b in zip(ps, ps[1:]))
        assert ps[0] == 1.0
