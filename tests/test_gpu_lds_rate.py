"""The LDS increment-rate measurement (bns_lds_increment_rate), the reference
that reports on the counting step use: it runs, returns a positive rate, and
the per-clock figure agrees with it (one increment per lane per cycle is the
most a compute unit's LDS could take: 64 per compute unit per cycle)."""

import pytest

pytestmark = pytest.mark.gpu


def test_lds_increment_rate():
    import paper_2212_04259_amd as b
    b.load()
    print("lds increment rate", flush=True)
    per_s, per_cu_clk = b.bns_lds_increment_rate(0)
    assert per_s > 0.0
    assert 0.5 < per_cu_clk <= 64.0, per_cu_clk
    again, _ = b.bns_lds_increment_rate(0)
    assert 0.5 < again / per_s < 2.0
