"""Python access to the C oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: plain, slow, single-threaded FP64 reference of the
G^2 CI test and PC-stable step 1.  Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import this package; the product library
never uses it.  It shares no code with the GPU path.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# BNS_ORACLE_LIB points the wrapper at another build of oracle.c (the pin
# suite uses it to run its checks against deliberately broken copies).
_LIB = os.environ.get("BNS_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

CI_FN = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                         ctypes.POINTER(ctypes.c_int32), ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_gamma_q.restype = ctypes.c_double
        L.orc_gamma_q.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_ci_test.restype = ctypes.c_int
        L.orc_ci_test.argtypes = [u8p, ctypes.c_int64, ctypes.c_int32, u8p, ctypes.c_int32,
                                  ctypes.c_int32, i32p, ctypes.c_int32, i64p, dp, i64p, dp]
        L.orc_ci_test_ex.restype = ctypes.c_int
        L.orc_ci_test_ex.argtypes = [u8p, ctypes.c_int64, ctypes.c_int32, u8p, ctypes.c_int32,
                                     ctypes.c_int32, i32p, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, i64p, dp, i64p, dp]
        L.orc_pc_skeleton_ex.restype = ctypes.c_void_p
        L.orc_pc_skeleton_ex.argtypes = [u8p, ctypes.c_int64, ctypes.c_int32, u8p, ctypes.c_double,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.orc_pc_skeleton.restype = ctypes.c_void_p
        L.orc_pc_skeleton.argtypes = [u8p, ctypes.c_int64, ctypes.c_int32, u8p, ctypes.c_double,
                                      ctypes.c_int32]
        L.orc_pc_skeleton_cb.restype = ctypes.c_void_p
        L.orc_pc_skeleton_cb.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_int32, CI_FN,
                                         ctypes.c_void_p]
        for name, res in [("orc_result_status", ctypes.c_int32), ("orc_result_n_vars", ctypes.c_int32),
                          ("orc_result_n_depths", ctypes.c_int32),
                          ("orc_result_knife_edges", ctypes.c_int64),
                          ("orc_result_min_gap", ctypes.c_double),
                          ("orc_result_pool_len", ctypes.c_int64)]:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = [ctypes.c_void_p]
        for name in ("orc_result_tests", "orc_result_removed"):
            f = getattr(L, name)
            f.restype = ctypes.c_int64
            f.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.orc_result_export.restype = None
        L.orc_result_export.argtypes = [ctypes.c_void_p, u8p, i32p, i32p]
        L.orc_result_pool.restype = None
        L.orc_result_pool.argtypes = [ctypes.c_void_p, i32p]
        L.orc_result_free.restype = None
        L.orc_result_free.argtypes = [ctypes.c_void_p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def gamma_q(a: float, x: float) -> float:
    """Regularised upper incomplete gamma Q(a, x)."""
    return float(lib().orc_gamma_q(float(a), float(x)))


def chi2_sf(stat: float, df: int) -> float:
    return 1.0 if df == 0 else gamma_q(0.5 * df, 0.5 * stat)


def _check_data(data, cards):
    data = np.ascontiguousarray(data, dtype=np.uint8)
    cards = np.ascontiguousarray(cards, dtype=np.uint8)
    if data.ndim != 2 or cards.shape != (data.shape[0],):
        raise ValueError("data must be uint8 [n_vars][n_samples] and cards uint8 [n_vars]")
    return data, cards


STAT_G2, STAT_X2 = 0, 1
DF_DECLARED, DF_ADJUSTED = 0, 1


def ci_test(data, cards, x: int, y: int, z=(), return_counts: bool = False, statistic: int = 0,
            df_rule: int = 0):
    """Test of I(x, y | z) with G^2 (statistic 0) or Pearson's X^2 (1), df
    from the declared cards (df_rule 0) or adjusted for empty rows, columns and
    strata (1).  Returns (stat, df, p) or (stat, df, p, counts)."""
    data, cards = _check_data(data, cards)
    n, m = data.shape
    z = np.ascontiguousarray(list(z), dtype=np.int32)
    T = 1
    if return_counts:
        if not all(0 <= v < n for v in [x, y] + z.tolist()):
            raise ValueError("variable index out of range")
        T = int(cards[x]) * int(cards[y]) * int(np.prod([int(cards[v]) for v in z], dtype=np.int64))
    counts = np.zeros(T, dtype=np.int64)
    g2 = ctypes.c_double()
    df = ctypes.c_int64()
    p = ctypes.c_double()
    rc = lib().orc_ci_test_ex(_ptr(data, ctypes.c_uint8), m, n, _ptr(cards, ctypes.c_uint8), x, y,
                              _ptr(z, ctypes.c_int32) if len(z) else None, len(z), int(statistic),
                              int(df_rule), _ptr(counts, ctypes.c_int64) if return_counts else None,
                              ctypes.byref(g2), ctypes.byref(df), ctypes.byref(p))
    if rc != 0:
        raise ValueError(f"orc_ci_test failed with {rc}")
    if return_counts:
        return g2.value, df.value, p.value, counts
    return g2.value, df.value, p.value


@dataclass
class SkeletonResult:
    adj: np.ndarray                  # uint8 [n][n]
    depth: np.ndarray                # int32 [n][n], removal depth or -1
    sepsets: dict                    # (i, j) with i < j -> tuple of ascending ids
    tests: list                      # tests run per depth
    removed: list                    # edges removed per depth
    knife_edges: int = 0
    min_gap: float = float("inf")
    extra: dict = field(default_factory=dict)

    @property
    def n_depths(self) -> int:
        return len(self.tests)

    def edges(self):
        n = self.adj.shape[0]
        return [(i, j) for i in range(n) for j in range(i + 1, n) if self.adj[i, j]]


def _collect(res_ptr) -> SkeletonResult:
    L = lib()
    try:
        st = L.orc_result_status(res_ptr)
        if st != 0:
            raise ValueError(f"oracle PC-stable failed with status {st}")
        n = L.orc_result_n_vars(res_ptr)
        adj = np.zeros((n, n), dtype=np.uint8)
        depth = np.zeros((n, n), dtype=np.int32)
        off = np.zeros((n, n), dtype=np.int32)
        L.orc_result_export(res_ptr, _ptr(adj, ctypes.c_uint8), _ptr(depth, ctypes.c_int32),
                            _ptr(off, ctypes.c_int32))
        plen = L.orc_result_pool_len(res_ptr)
        pool = np.zeros(max(plen, 1), dtype=np.int32)
        L.orc_result_pool(res_ptr, _ptr(pool, ctypes.c_int32))
        sep = {}
        ii, jj = np.nonzero(np.triu(depth >= 0, 1))
        for i, j in zip(ii.tolist(), jj.tolist()):
            d = int(depth[i, j])
            o = int(off[i, j])
            sep[(i, j)] = tuple(int(v) for v in pool[o:o + d])
        nd = L.orc_result_n_depths(res_ptr)
        tests = [int(L.orc_result_tests(res_ptr, d)) for d in range(nd)]
        removed = [int(L.orc_result_removed(res_ptr, d)) for d in range(nd)]
        return SkeletonResult(adj=adj, depth=depth, sepsets=sep, tests=tests, removed=removed,
                              knife_edges=int(L.orc_result_knife_edges(res_ptr)),
                              min_gap=float(L.orc_result_min_gap(res_ptr)))
    finally:
        L.orc_result_free(res_ptr)


def pc_skeleton(data, cards, alpha: float = 0.05, max_depth: int = -1, statistic: int = 0,
                df_rule: int = 0) -> SkeletonResult:
    """PC-stable step 1 with the G^2 test (Algorithm 1 with Section IV-C
    grouping); statistic and df_rule as in ci_test."""
    data, cards = _check_data(data, cards)
    n, m = data.shape
    r = lib().orc_pc_skeleton_ex(_ptr(data, ctypes.c_uint8), m, n, _ptr(cards, ctypes.c_uint8),
                                 float(alpha), int(max_depth), int(statistic), int(df_rule))
    if not r:
        raise MemoryError("oracle allocation failed")
    return _collect(r)


def pc_skeleton_cb(n: int, pvalue_fn, alpha: float = 0.05, max_depth: int = -1) -> SkeletonResult:
    """PC-stable step 1 with a caller-supplied CI p-value source
    ``pvalue_fn(x, y, S_tuple) -> float``."""
    def _tramp(_user, x, y, s, d):
        return float(pvalue_fn(int(x), int(y), tuple(int(s[k]) for k in range(d))))

    cb = CI_FN(_tramp)
    r = lib().orc_pc_skeleton_cb(int(n), float(alpha), int(max_depth), cb, None)
    if not r:
        raise MemoryError("oracle allocation failed")
    return _collect(r)
