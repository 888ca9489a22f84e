"""The oracle's pins must catch plausible mistakes.

Each case below plants one mistake in a copy of oracle.c (on the CPU, in a
temporary directory), builds it, and runs the pin suite against that build
through BNS_ORACLE_LIB.  Every mutant must make at least one pin fail; the
unmodified source must pass them all.
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
PINS = ["tests/test_oracle_ci.py", "tests/test_oracle_pvalue.py", "tests/test_oracle_pc.py",
        "tests/test_oracle_stats.py"]

MUTANTS = {
    "transposed_cell_index": ("N[cx[s] + rx * (cy[s] + ry * zc)]", "N[cx[s] + ry * (cy[s] + rx * zc)]"),
    "dropped_factor_two": ("G2 = 2.0 * sum;", "G2 = sum;"),
    "inverted_log_ratio": ("log((double)num / (double)den)", "log((double)den / (double)num)"),
    "df_without_strata": ("(rx - 1) * (ry - 1) * nstrata;", "(rx - 1) * (ry - 1);"),
    "tie_counts_as_independent": ("if (pv > alpha) {", "if (pv >= alpha) {"),
    "side_b_first": ("rc = test_side(r, i, j, candA, pA, d, alpha, fn, user, idx, S);\n"
                     "                    if (rc == 0) rc = test_side(r, i, j, candB, pB, d, alpha, fn, user, idx, S);",
                     "rc = test_side(r, i, j, candB, pB, d, alpha, fn, user, idx, S);\n"
                     "                    if (rc == 0) rc = test_side(r, i, j, candA, pA, d, alpha, fn, user, idx, S);"),
    "series_index_off_by_one": ("term *= x / (a + n);", "term *= x / (a + n + 1);"),
    "cfrac_step": ("b += 2.0;", "b += 1.0;"),
    "marginal_ignores_stratum": ("Nxz[xv + rx * zc] += c;", "Nxz[xv] += c;"),
    "stop_rule_strict": ("deg[i] - 1 >= d || deg[j] - 1 >= d", "deg[i] - 1 > d || deg[j] - 1 > d"),
    "no_snapshot": ("if (snap[i * n + k] != j) candA[pA++] = snap[i * n + k];",
                    "if (snap[i * n + k] != j && r->adj[i * n + snap[i * n + k]]) candA[pA++] = snap[i * n + k];"),
    "z_radix_wrong": ("mult *= cards[z[k]];", "mult *= rx;"),
    "knife_edges_never_counted": ("if (gap < 1e-9) r->knife += 1;", "if (gap < 0.0) r->knife += 1;"),
    "gap_measured_on_complement": ("double gap = fabs(pv - alpha);", "double gap = fabs((1.0 - pv) - alpha);"),
    "x2_not_squared": ("sum += diff * diff / E;", "sum += fabs(diff) / E;"),
    "x2_smoothed_expectation": ("sum += diff * diff / E;", "sum += diff * diff / (E + 0.5);"),
    "adjusted_df_keeps_empty_rows": ("a += Nxz[xv + rx * zc] > 0;", "a += 1;"),
    "adjusted_df_counts_empty_strata": ("            if (Nz[zc] == 0) continue;\n            int64_t a = 0, b = 0;",
                                        "            int64_t a = 0, b = 0;"),
}


def _run_pins(lib_path):
    env = dict(os.environ, BNS_ORACLE_LIB=lib_path)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] + PINS,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode


def _build(tmp_path, src_text, name):
    c = tmp_path / f"{name}.c"
    c.write_text(src_text)
    so = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-I", os.path.dirname(SRC),
                           "-o", str(so), str(c), "-lm"])
    return str(so)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    so = _build(tmp_path, src.replace(old, new), name)
    assert _run_pins(so) != 0, f"pins did not catch mutant {name}"


def test_unmodified_source_passes(tmp_path):
    so = _build(tmp_path, open(SRC).read(), "clean")
    assert _run_pins(so) == 0


# Mistakes planted in copies of the orientation oracle (oracle/orient.py),
# caught by tests/test_oracle_orient.py.
ORIENT_SRC = os.path.join(ROOT, "oracle", "orient.py")
ORIENT_MUTANTS = {
    "collider_when_in_sepset": ("if z not in sepsets[(min(x, y), max(x, y))]:",
                                "if z in sepsets[(min(x, y), max(x, y))]:"),
    "triples_ignore_adjacency": ("                if adj[x, y]:\n                    continue\n", ""),
    "r1_without_nonadjacency": ("r1 = D[:, a] & ~adj[:, b]", "r1 = D[:, a].copy()"),
    "r2_reversed": ("if (D[a, :] & D[:, b]).any():", "if (D[:, a] & D[b, :]).any():"),
    "r3_dropped": ("            if any(not adj[c, d] for i, c in enumerate(cs) for d in cs[i + 1:]):\n"
                   "                found.add((a, b))\n", ""),
    "conflict_resolved_by_order": ("            if (b, a) not in found:\n                G[b, a] = 1",
                                   "            G[b, a] = 1"),
}


@pytest.mark.parametrize("name", sorted(ORIENT_MUTANTS))
def test_orient_mutant_is_caught(tmp_path, name):
    src = open(ORIENT_SRC).read()
    old, new = ORIENT_MUTANTS[name]
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    path = tmp_path / "orient_mut.py"
    path.write_text(src.replace(old, new))
    env = dict(os.environ, BNS_ORIENT_SRC=str(path))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "tests/test_oracle_orient.py"], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode != 0, f"pins did not catch orientation mutant {name}"
