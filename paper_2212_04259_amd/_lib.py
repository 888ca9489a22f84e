"""ctypes binding of libbns.so (include/bns.h).

Argument marshalling only: every step of the CI tests and of the skeleton
search runs in the library's gfx950 kernels.  The library must be built
(``python -m paper_2212_04259_amd.build``); importing this module without it
raises, there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbns.so")

BNS_OK = 0
BNS_FORM_BATCHED, BNS_FORM_PLAIN, BNS_FORM_EDGE = 0, 1, 2
BNS_PREC_FP32_RECHECK, BNS_PREC_FP64 = 0, 1
BNS_CI_INDEPENDENT, BNS_CI_RECHECKED = 1, 2
BNS_STAT_G2, BNS_STAT_X2 = 0, 1
BNS_DF_DECLARED, BNS_DF_ADJUSTED = 0, 1
BNS_DEPTH0_AUTO, BNS_DEPTH0_TESTS, BNS_DEPTH0_PAIRS = 0, 1, 2
BNS_DEPTH1_AUTO, BNS_DEPTH1_TESTS, BNS_DEPTH1_GRAM = 0, 1, 2
BNS_GROUP_AUTO, BNS_GROUP_TEST, BNS_GROUP_EDGE = 0, 1, 2
STATUS_NAMES = {0: "BNS_OK", 1: "BNS_E_INVALID_ARG", 2: "BNS_E_VALUE_RANGE",
                3: "BNS_E_TABLE_TOO_LARGE", 4: "BNS_E_NOMEM", 5: "BNS_E_DEVICE",
                6: "BNS_E_INTERNAL"}

# Every symbol include/bns.h declares.
EXPORTS = [
    "bns_options_default", "bns_last_error", "bns_dataset_create", "bns_dataset_wrap_device",
    "bns_dataset_free", "bns_ci_batch", "bns_pc_skeleton", "bns_pc_skeleton_dataset",
    "bns_pc_skeleton_batch", "bns_skeleton_n_vars", "bns_skeleton_adjacency",
    "bns_skeleton_sepset", "bns_skeleton_removals", "bns_skeleton_stats", "bns_skeleton_free",
    "bns_autotune", "bns_ci_batch_noalloc", "bns_skeleton_orient", "bns_skeleton_create",
    "bns_ci_pairs", "bns_lds_increment_rate",
]
NOALLOC_SCRATCH_BYTES = 16 << 20


class BnsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class bns_options(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("recheck_band", ctypes.c_double), ("lds_bytes", ctypes.c_int32),
                ("wg_per_cu", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("split_min_samples", ctypes.c_int32),
                ("units_per_group", ctypes.c_int32), ("test_group", ctypes.c_int32),
                ("max_replicas", ctypes.c_int32), ("tickets_per_grab", ctypes.c_int32),
                ("ticket_runs", ctypes.c_int32), ("wave_depths", ctypes.c_uint32),
                ("block_depths", ctypes.c_uint32), ("report_errors", ctypes.c_int32),
                ("workspace_mb", ctypes.c_int32), ("statistic", ctypes.c_int32),
                ("df_rule", ctypes.c_int32), ("depth0", ctypes.c_int32),
                ("round_tests", ctypes.c_int32), ("depth1", ctypes.c_int32),
                ("group_tests", ctypes.c_int32),
                ("stream", ctypes.c_void_p)]


class bns_ci_test(ctypes.Structure):
    _fields_ = [("x", ctypes.c_int32), ("y", ctypes.c_int32), ("n_z", ctypes.c_int32),
                ("z_offset", ctypes.c_int32)]


class bns_depth_stats(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("test_group", ctypes.c_int32),
                ("edges", ctypes.c_int64), ("tests_required", ctypes.c_int64),
                ("tests_executed", ctypes.c_int64), ("removed", ctypes.c_int64),
                ("rechecks", ctypes.c_int64), ("tickets", ctypes.c_int64),
                ("operand_bytes", ctypes.c_double), ("kernel_seconds", ctypes.c_double),
                ("span_seconds", ctypes.c_double), ("err_tests", ctypes.c_int64),
                ("err_flips", ctypes.c_int64), ("err_max", ctypes.c_double),
                ("err_p50", ctypes.c_double), ("err_p99", ctypes.c_double),
                ("chunks", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("chunk_samples", ctypes.c_int64)]


_lib = None


def load():
    """Loads libbns.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2212_04259_amd.build")
    # torch bundles its own HIP runtime.  Loading torch first lets libbns.so
    # bind to that same runtime (matching SONAME), so device pointers and
    # streams are shared and the process holds a single HIP runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    L.bns_options_default.restype = None
    L.bns_options_default.argtypes = [P(bns_options)]
    L.bns_last_error.restype = ctypes.c_char_p
    L.bns_last_error.argtypes = []
    L.bns_dataset_create.restype = i32
    L.bns_dataset_create.argtypes = [vp, i64, i32, vp, P(vp)]
    L.bns_dataset_wrap_device.restype = i32
    L.bns_dataset_wrap_device.argtypes = [vp, i64, i64, i32, vp, P(vp)]
    L.bns_dataset_free.restype = None
    L.bns_dataset_free.argtypes = [vp]
    L.bns_ci_batch.restype = i32
    L.bns_ci_batch.argtypes = [vp, vp, i64, vp, i64, dbl, P(bns_options), vp, vp, vp, vp, vp, vp]
    L.bns_ci_batch_noalloc.restype = i32
    L.bns_ci_batch_noalloc.argtypes = [vp, vp, i64, vp, i64, dbl, P(bns_options), vp, vp, vp, vp]
    L.bns_pc_skeleton.restype = i32
    L.bns_pc_skeleton.argtypes = [vp, i64, i32, vp, dbl, i32, P(bns_options), P(vp)]
    L.bns_pc_skeleton_dataset.restype = i32
    L.bns_pc_skeleton_dataset.argtypes = [vp, dbl, i32, P(bns_options), P(vp)]
    L.bns_pc_skeleton_batch.restype = i32
    L.bns_pc_skeleton_batch.argtypes = [vp, i32, vp, vp, P(bns_options), vp]
    L.bns_autotune.restype = i32
    L.bns_autotune.argtypes = [vp, i32, vp, vp, P(bns_options), i32, P(bns_options)]
    L.bns_skeleton_n_vars.restype = i32
    L.bns_skeleton_n_vars.argtypes = [vp]
    L.bns_skeleton_adjacency.restype = i32
    L.bns_skeleton_adjacency.argtypes = [vp, vp]
    L.bns_skeleton_sepset.restype = i32
    L.bns_skeleton_sepset.argtypes = [vp, i32, i32, vp, i32, P(i32), P(i32)]
    L.bns_skeleton_removals.restype = i32
    L.bns_skeleton_removals.argtypes = [vp, vp, vp, vp, i64, P(i64)]
    L.bns_skeleton_stats.restype = i32
    L.bns_skeleton_stats.argtypes = [vp, P(bns_depth_stats), i32, P(i32)]
    L.bns_ci_pairs.restype = i32
    L.bns_ci_pairs.argtypes = [vp, dbl, P(bns_options), vp, vp, vp, vp]
    L.bns_skeleton_create.restype = i32
    L.bns_skeleton_create.argtypes = [i32, vp, vp, vp, vp, i64, P(vp)]
    L.bns_skeleton_orient.restype = i32
    L.bns_skeleton_orient.argtypes = [vp, vp]
    L.bns_lds_increment_rate.restype = i32
    L.bns_lds_increment_rate.argtypes = [i32, P(dbl), P(dbl)]
    L.bns_skeleton_free.restype = None
    L.bns_skeleton_free.argtypes = [vp]
    _lib = L
    return L


def _check(st: int):
    if st != BNS_OK:
        raise BnsError(st, load().bns_last_error().decode())


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def bns_lds_increment_rate(device: int = 0):
    """(increments per second, per compute unit per clock) of the device's LDS
    (bns_lds_increment_rate)."""
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(load().bns_lds_increment_rate(int(device), ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def bns_options_default(**kw) -> bns_options:
    o = bns_options()
    load().bns_options_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Dataset:
    """A bns_dataset handle (device-resident columns)."""

    def __init__(self, handle, n_vars, n_samples, keepalive=None):
        self.handle = handle
        self.n_vars = n_vars
        self.n_samples = n_samples
        self._keep = keepalive

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.bns_dataset_free(self.handle)
            self.handle = None


def bns_dataset_create(data: np.ndarray, cards: np.ndarray) -> Dataset:
    data = np.ascontiguousarray(data, dtype=np.uint8)
    cards = np.ascontiguousarray(cards, dtype=np.uint8)
    h = ctypes.c_void_p()
    _check(load().bns_dataset_create(_ptr(data), data.shape[1], data.shape[0], _ptr(cards),
                                     ctypes.byref(h)))
    return Dataset(h, data.shape[0], data.shape[1])


def bns_dataset_wrap_device(tensor, n_samples: int, cards: np.ndarray) -> Dataset:
    """Wraps a device tensor uint8 [n_vars][ld] (torch) without copying."""
    cards = np.ascontiguousarray(cards, dtype=np.uint8)
    n, ld = int(tensor.shape[0]), int(tensor.stride(0))
    h = ctypes.c_void_p()
    _check(load().bns_dataset_wrap_device(ctypes.c_void_p(tensor.data_ptr()), ld, n_samples, n,
                                          _ptr(cards), ctypes.byref(h)))
    return Dataset(h, n, n_samples, keepalive=tensor)


def bns_ci_batch(ds: Dataset, tests, alpha: float = 0.05, options: bns_options | None = None,
                 want_tables: bool = False, cards=None):
    """Runs tests given as (x, y, z_tuple).  Returns a dict of numpy arrays
    g2, df, p, flags (and tables: list of int32 arrays when want_tables)."""
    n = len(tests)
    arr = (bns_ci_test * max(n, 1))()
    zs = []
    for t, (x, y, z) in enumerate(tests):
        arr[t].x, arr[t].y, arr[t].n_z, arr[t].z_offset = int(x), int(y), len(z), len(zs)
        zs.extend(int(v) for v in z)
    zpool = np.asarray(zs if zs else [0], dtype=np.int32)
    g2 = np.zeros(max(n, 1), dtype=np.float64)
    df = np.zeros(max(n, 1), dtype=np.int64)
    p = np.zeros(max(n, 1), dtype=np.float64)
    flags = np.zeros(max(n, 1), dtype=np.int32)
    tabs = offs = None
    sizes = None
    if want_tables:
        if cards is None:
            raise ValueError("want_tables needs the dataset's cards")
        sizes = [int(cards[x]) * int(cards[y]) * int(np.prod([int(cards[v]) for v in z]))
                 for (x, y, z) in tests]
        offs = np.zeros(max(n, 1), dtype=np.int64)
        if n:
            offs[:n] = np.concatenate([[0], np.cumsum(sizes)[:-1]])
        tabs = np.zeros(max(int(sum(sizes)), 1), dtype=np.int32)
    o = options if options is not None else bns_options_default()
    _check(load().bns_ci_batch(ds.handle, ctypes.cast(arr, ctypes.c_void_p), n, _ptr(zpool),
                               len(zs), float(alpha), ctypes.byref(o), _ptr(g2), _ptr(df), _ptr(p),
                               _ptr(flags), _ptr(tabs), _ptr(offs)))
    out = dict(g2=g2[:n], df=df[:n], p=p[:n], flags=flags[:n])
    if want_tables:
        out["tables"] = [tabs[offs[t]:offs[t] + sizes[t]] for t in range(n)]
    return out


def bns_ci_pairs(ds: Dataset, alpha: float = 0.05, options: bns_options | None = None):
    """Every pairwise marginal test of the dataset (bns_ci_pairs).  Returns a
    dict of numpy arrays stat, df, p, flags in the order of the pairs i < j,
    and pairs: the (i, j) of each entry."""
    n = ds.n_vars
    npairs = n * (n - 1) // 2
    stat = np.zeros(max(npairs, 1), dtype=np.float64)
    df = np.zeros(max(npairs, 1), dtype=np.int64)
    p = np.zeros(max(npairs, 1), dtype=np.float64)
    flags = np.zeros(max(npairs, 1), dtype=np.int32)
    o = options if options is not None else bns_options_default()
    _check(load().bns_ci_pairs(ds.handle, float(alpha), ctypes.byref(o), _ptr(stat), _ptr(df), _ptr(p),
                               _ptr(flags)))
    ii, jj = np.triu_indices(n, 1)
    return dict(stat=stat[:npairs], df=df[:npairs], p=p[:npairs], flags=flags[:npairs],
                pairs=list(zip(ii.tolist(), jj.tolist())))


def bns_ci_batch_noalloc(ds: Dataset, tests, alpha: float = 0.05, options: bns_options | None = None):
    """bns_ci_batch through the allocation-free entry point (no table output).
    Returns a dict of numpy arrays g2, df, p, flags."""
    n = len(tests)
    arr = (bns_ci_test * max(n, 1))()
    zs = []
    for t, (x, y, z) in enumerate(tests):
        arr[t].x, arr[t].y, arr[t].n_z, arr[t].z_offset = int(x), int(y), len(z), len(zs)
        zs.extend(int(v) for v in z)
    zpool = np.asarray(zs if zs else [0], dtype=np.int32)
    g2 = np.zeros(max(n, 1), dtype=np.float64)
    df = np.zeros(max(n, 1), dtype=np.int64)
    p = np.zeros(max(n, 1), dtype=np.float64)
    flags = np.zeros(max(n, 1), dtype=np.int32)
    o = options if options is not None else bns_options_default()
    _check(load().bns_ci_batch_noalloc(ds.handle, ctypes.cast(arr, ctypes.c_void_p), n, _ptr(zpool),
                                       len(zs), float(alpha), ctypes.byref(o), _ptr(g2), _ptr(df),
                                       _ptr(p), _ptr(flags)))
    return dict(g2=g2[:n], df=df[:n], p=p[:n], flags=flags[:n])


@dataclass
class Skeleton:
    adj: np.ndarray
    depth: np.ndarray
    sepsets: dict
    stats: list = field(default_factory=list)
    cpdag: np.ndarray | None = None   # int8 marks of bns_skeleton_orient (when asked for)

    def edges(self):
        n = self.adj.shape[0]
        return [(i, j) for i in range(n) for j in range(i + 1, n) if self.adj[i, j]]


def _collect(h, orient: bool = False) -> Skeleton:
    L = load()
    try:
        n = L.bns_skeleton_n_vars(h)
        adj = np.zeros((n, n), dtype=np.uint8)
        _check(L.bns_skeleton_adjacency(h, _ptr(adj)))
        depth = np.zeros((n, n), dtype=np.int32)
        off = np.zeros((n, n), dtype=np.int64)
        plen = ctypes.c_int64()
        _check(L.bns_skeleton_removals(h, _ptr(depth), _ptr(off), None, 0, ctypes.byref(plen)))
        pool = np.zeros(max(plen.value, 1), dtype=np.int32)
        _check(L.bns_skeleton_removals(h, None, None, _ptr(pool), plen.value, ctypes.byref(plen)))
        sep = {}
        ii, jj = np.nonzero(np.triu(depth >= 0, 1))
        for i, j in zip(ii.tolist(), jj.tolist()):
            d, o = int(depth[i, j]), int(off[i, j])
            sep[(i, j)] = tuple(int(v) for v in pool[o:o + d])
        nd = ctypes.c_int32()
        _check(L.bns_skeleton_stats(h, None, 0, ctypes.byref(nd)))
        st = (bns_depth_stats * max(nd.value, 1))()
        _check(L.bns_skeleton_stats(h, st, nd.value, ctypes.byref(nd)))
        stats = [{f: getattr(st[d], f) for f, _ in bns_depth_stats._fields_} for d in range(nd.value)]
        cp = None
        if orient:
            cp = np.zeros((n, n), dtype=np.int8)
            _check(L.bns_skeleton_orient(h, _ptr(cp)))
        return Skeleton(adj=adj, depth=depth, sepsets=sep, stats=stats, cpdag=cp)
    finally:
        L.bns_skeleton_free(h)


def bns_pc_skeleton(data: np.ndarray, cards: np.ndarray, alpha: float = 0.05, max_depth: int = -1,
                    options: bns_options | None = None, orient: bool = False) -> Skeleton:
    data = np.ascontiguousarray(data, dtype=np.uint8)
    cards = np.ascontiguousarray(cards, dtype=np.uint8)
    o = options if options is not None else bns_options_default()
    h = ctypes.c_void_p()
    _check(load().bns_pc_skeleton(_ptr(data), data.shape[1], data.shape[0], _ptr(cards),
                                  float(alpha), int(max_depth), ctypes.byref(o), ctypes.byref(h)))
    return _collect(h, orient)


def bns_pc_skeleton_dataset(ds: Dataset, alpha: float = 0.05, max_depth: int = -1,
                            options: bns_options | None = None, orient: bool = False) -> Skeleton:
    o = options if options is not None else bns_options_default()
    h = ctypes.c_void_p()
    _check(load().bns_pc_skeleton_dataset(ds.handle, float(alpha), int(max_depth),
                                          ctypes.byref(o), ctypes.byref(h)))
    return _collect(h, orient)


def bns_autotune(datasets, alphas, max_depths, base: bns_options | None = None,
                 trials: int = 0) -> bns_options:
    """Launch options for the batched search of these datasets, chosen by
    timing trial searches in the library (cached per device and workload)."""
    k = len(datasets)
    hs = (ctypes.c_void_p * k)(*[d.handle for d in datasets])
    al = np.ascontiguousarray(alphas, dtype=np.float64)
    md = np.ascontiguousarray(max_depths, dtype=np.int32)
    b = base if base is not None else bns_options_default()
    out = bns_options()
    _check(load().bns_autotune(ctypes.cast(hs, ctypes.c_void_p), k, _ptr(al), _ptr(md),
                               ctypes.byref(b), int(trials), ctypes.byref(out)))
    return out


def bns_pc_skeleton_batch(datasets, alphas, max_depths, options: bns_options | None = None,
                          orient: bool = False):
    k = len(datasets)
    hs = (ctypes.c_void_p * k)(*[d.handle for d in datasets])
    al = np.ascontiguousarray(alphas, dtype=np.float64)
    md = np.ascontiguousarray(max_depths, dtype=np.int32)
    outs = (ctypes.c_void_p * k)()
    o = options if options is not None else bns_options_default()
    _check(load().bns_pc_skeleton_batch(ctypes.cast(hs, ctypes.c_void_p), k, _ptr(al), _ptr(md),
                                        ctypes.byref(o), ctypes.cast(outs, ctypes.c_void_p)))
    return [_collect(ctypes.c_void_p(outs[i]), orient) for i in range(k)]


def skeleton_handle(ds: Dataset, alpha: float, max_depth: int, options: bns_options):
    """Runs bns_pc_skeleton_dataset and returns the raw result handle (the
    caller frees it with free_skeleton); used where result conversion must
    stay outside a timed region."""
    h = ctypes.c_void_p()
    _check(load().bns_pc_skeleton_dataset(ds.handle, float(alpha), int(max_depth),
                                          ctypes.byref(options), ctypes.byref(h)))
    return h


def skeleton_batch_handles(datasets, alphas, max_depths, options: bns_options):
    k = len(datasets)
    hs = (ctypes.c_void_p * k)(*[d.handle for d in datasets])
    al = np.ascontiguousarray(alphas, dtype=np.float64)
    md = np.ascontiguousarray(max_depths, dtype=np.int32)
    outs = (ctypes.c_void_p * k)()
    _check(load().bns_pc_skeleton_batch(ctypes.cast(hs, ctypes.c_void_p), k, _ptr(al), _ptr(md),
                                        ctypes.byref(options), ctypes.cast(outs, ctypes.c_void_p)))
    return [ctypes.c_void_p(outs[i]) for i in range(k)]


def bns_orient(adj: np.ndarray, sepsets: dict) -> np.ndarray:
    """CPDAG marks (bns_skeleton_orient) of a skeleton given on the host:
    adj (n x n 0/1) and sepsets {(i, j): members} of every removed pair."""
    adj = np.ascontiguousarray(adj, dtype=np.uint8)
    n = adj.shape[0]
    depth = np.full((n, n), -1, dtype=np.int32)
    off = np.full((n, n), -1, dtype=np.int64)
    pool = []
    for (i, j), S in sorted(sepsets.items()):
        depth[i, j] = depth[j, i] = len(S)
        off[i, j] = off[j, i] = len(pool)
        pool.extend(int(v) for v in S)
    pa = np.asarray(pool if pool else [0], dtype=np.int32)
    h = ctypes.c_void_p()
    L = load()
    _check(L.bns_skeleton_create(n, _ptr(adj), _ptr(depth), _ptr(off), _ptr(pa), len(pool), ctypes.byref(h)))
    try:
        cp = np.zeros((n, n), dtype=np.int8)
        _check(L.bns_skeleton_orient(h, _ptr(cp)))
        return cp
    finally:
        L.bns_skeleton_free(h)


def free_skeleton(h) -> None:
    load().bns_skeleton_free(h)


def collect(h, orient: bool = False) -> Skeleton:
    """Converts a raw result handle into a Skeleton and frees the handle."""
    return _collect(h, orient)
