"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments on the host before any device work (no GPU needed)."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bns.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bns_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def bns():
    import paper_2212_04259_amd as b
    b.load()
    return b


def test_every_declared_symbol_is_exported(bns):
    L = bns.load()
    decl = _declared()
    assert decl, "no declarations parsed"
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(bns.EXPORTS) == decl


def test_options_defaults(bns):
    o = bns.bns_options_default()
    assert o.form == bns.BNS_FORM_BATCHED
    assert o.precision == bns.BNS_PREC_FP32_RECHECK
    assert o.recheck_band == 1e-3
    assert o.use_graph == 1 and o.timing == 0
    assert o.wave_depths == 0 and o.block_depths == 0 and o.group_tests == 0 and o.round_tests == 0
    assert o.report_errors == 0 and o.workspace_mb == 0
    assert o.statistic == bns.BNS_STAT_G2 and o.df_rule == bns.BNS_DF_DECLARED
    assert o.depth0 == bns.BNS_DEPTH0_AUTO and o.depth1 == bns.BNS_DEPTH1_AUTO


@pytest.mark.parametrize("data,cards,alpha,maxd,msg", [
    (np.zeros((3, 10), np.uint8), np.array([2, 2, 0], np.uint8), 0.05, -1, "BNS_E_INVALID_ARG"),
    (np.full((3, 10), 3, np.uint8), np.array([2, 2, 2], np.uint8), 0.05, -1, "BNS_E_VALUE_RANGE"),
    (np.zeros((3, 10), np.uint8), np.array([2, 2, 2], np.uint8), 0.0, -1, "BNS_E_INVALID_ARG"),
    (np.zeros((3, 10), np.uint8), np.array([2, 2, 2], np.uint8), 1.0, -1, "BNS_E_INVALID_ARG"),
    (np.zeros((3, 10), np.uint8), np.array([2, 2, 2], np.uint8), 0.05, -2, "BNS_E_INVALID_ARG"),
    (np.zeros((1, 10), np.uint8), np.array([2], np.uint8), 0.05, -1, "BNS_E_INVALID_ARG"),
])
def test_host_validation(bns, data, cards, alpha, maxd, msg):
    with pytest.raises(bns.BnsError) as ei:
        bns.bns_pc_skeleton(data, cards, alpha, maxd)
    assert msg in str(ei.value)


def test_value_range_names_the_sample(bns):
    data = np.zeros((4, 100), np.uint8)
    data[2, 37] = 5
    with pytest.raises(bns.BnsError) as ei:
        bns.bns_pc_skeleton(data, np.array([2, 2, 3, 2], np.uint8))
    assert "variable 2" in str(ei.value) and "sample 37" in str(ei.value)


def test_bad_options_rejected(bns):
    o = bns.bns_options_default(form=7)
    with pytest.raises(bns.BnsError):
        bns.bns_pc_skeleton(np.zeros((3, 10), np.uint8), np.array([2, 2, 2], np.uint8), options=o)
    o = bns.bns_options_default()
    o.group_tests = 3
    with pytest.raises(bns.BnsError):
        bns.bns_pc_skeleton(np.zeros((3, 10), np.uint8), np.array([2, 2, 2], np.uint8), options=o)
    for bad in (dict(split_min_samples=-2), dict(units_per_group=-1), dict(units_per_group=5000),
                dict(test_group=3), dict(test_group=-1), dict(max_replicas=3),
                dict(max_replicas=128), dict(tickets_per_grab=9), dict(tickets_per_grab=-1),
                dict(ticket_runs=3), dict(ticket_runs=-1),
                dict(wave_depths=0b110, block_depths=0b011), dict(report_errors=2), dict(depth1=3), dict(depth1=-1),
                dict(report_errors=-1), dict(workspace_mb=-1), dict(statistic=2), dict(statistic=-1),
                dict(df_rule=2), dict(depth0=3), dict(depth0=-1), dict(round_tests=-1),
                dict(round_tests=65537), dict(form=3)):
        o = bns.bns_options_default(**bad)
        with pytest.raises(bns.BnsError, match="options"):
            bns.bns_pc_skeleton(np.zeros((3, 10), np.uint8), np.array([2, 2, 2], np.uint8),
                                options=o)


def test_null_handles(bns):
    L = bns.load()
    assert L.bns_skeleton_n_vars(None) == 0
    L.bns_skeleton_free(None)
    L.bns_dataset_free(None)
    assert L.bns_ci_batch(None, None, 0, None, 0, 0.05, None, None, None, None, None, None, None) == 1
    assert isinstance(L.bns_last_error(), bytes)
