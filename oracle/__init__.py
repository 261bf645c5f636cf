"""TEST INFRASTRUCTURE ONLY: Python access to the plain C oracle.

The oracle is a slow, serial CPU reference of frequent itemset mining by
Dynamic Itemset Counting (Algorithms 2-5 of the paper) plus independent
cross-checks (Apriori, exhaustive enumeration, depth-first enumeration over
transaction-id lists).  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import it; the GPU library never does, and this package
never imports the GPU library.

``build()`` compiles ``dic_oracle.c`` with gcc into ``liboracle.so`` beside it
(plain -O2, serial: the checker) and into ``liboracle_omp.so`` (-O3
-march=native -fopenmp: the same source with its count loop shared among
threads, timed as the benchmark's parallel CPU baseline; identical results).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dic_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_SO_OMP = os.path.join(_HERE, "liboracle_omp.so")
_lib = None
_lib_omp = None

OR_OK, OR_E_INVAL, OR_E_NOMEM, OR_E_RANGE = 0, -1, -2, -3


class OracleError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: oracle error {code}")
        self.code = code


class _Stop(ctypes.Structure):
    _fields_ = [("stop", ctypes.c_uint32), ("rows", ctypes.c_uint32), ("live", ctypes.c_uint64),
                ("promoted", ctypes.c_uint64), ("pruned", ctypes.c_uint64),
                ("generated", ctypes.c_uint64), ("solidified", ctypes.c_uint64)]


class _Stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in (
        "tau", "block", "stop_max", "stops", "tests", "peak_live", "n_frequent", "k_max",
        "known", "superset_prunes", "fullpass_promotions")]


TRACE_FIELDS = ("stop", "rows", "live", "promoted", "pruned", "generated", "solidified")


def build() -> str:
    """Compile the oracle (plain -O2, no target-specific flags) and its
    OpenMP build."""
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                           "-o", tmp, _SRC, "-lm"], cwd=_HERE)
    os.replace(tmp, _SO)
    build_parallel()
    return _SO


def build_parallel() -> str:
    """The same source with -O3 -march=native -fopenmp (the count loop over
    live candidates shared among threads)."""
    tmp = _SO_OMP + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-march=native", "-fopenmp", "-std=c11", "-Wall",
                           "-Wextra", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"], cwd=_HERE)
    os.replace(tmp, _SO_OMP)
    return _SO_OMP


def _declare(L):
    u64, u32, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
    pp = ctypes.POINTER(ctypes.c_void_p)
    L.oracle_threads.argtypes = [ctypes.c_int]
    L.oracle_threads.restype = ctypes.c_int
    L.oracle_dic_init.argtypes = [p, u64, u32, ctypes.c_double, u64, ctypes.c_int, ctypes.c_int,
                                  pp]
    for f in ("oracle_result_size", "oracle_result_trace_len"):
        getattr(L, f).restype = u64
        getattr(L, f).argtypes = [p]
    L.oracle_result_words.restype = u32
    L.oracle_result_words.argtypes = [p]
    L.oracle_result_masks.restype = p
    L.oracle_result_masks.argtypes = [p]
    L.oracle_result_counts.restype = p
    L.oracle_result_counts.argtypes = [p]
    L.oracle_result_stats.argtypes = [p, ctypes.POINTER(_Stats)]
    L.oracle_result_trace.restype = ctypes.POINTER(_Stop)
    L.oracle_result_trace.argtypes = [p]
    L.oracle_result_free.argtypes = [p]
    L.oracle_result_free.restype = None


def _load_parallel():
    global _lib_omp
    if _lib_omp is not None:
        return _lib_omp
    if not os.path.exists(_SO_OMP) or os.path.getmtime(_SO_OMP) < os.path.getmtime(_SRC):
        build_parallel()
    L = ctypes.CDLL(_SO_OMP)
    _declare(L)
    _lib_omp = L
    return L


def dic_parallel(rows, m: int, minsup: float, M: int, threads: int) -> tuple:
    """oracle.dic from the OpenMP build with the given thread count; returns
    (Result, threads used)."""
    L = _load_parallel()
    used = L.oracle_threads(int(threads))
    r = _rows(rows)
    h = ctypes.c_void_p()
    rc = L.oracle_dic_init(r.ctypes.data, r.shape[0], int(m), float(minsup), int(M), 0, 0,
                           ctypes.byref(h))
    if rc:
        raise OracleError(rc, "oracle_dic (OpenMP build)")
    return _collect(L, h, "dic"), used


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build()
    L = ctypes.CDLL(_SO)
    u64, u32, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
    pp = ctypes.POINTER(ctypes.c_void_p)
    L.oracle_tau.argtypes = [ctypes.c_double, u64, ctypes.POINTER(u64)]
    L.oracle_dic.argtypes = [p, u64, u32, ctypes.c_double, u64, ctypes.c_int, pp]
    L.oracle_dic_init.argtypes = [p, u64, u32, ctypes.c_double, u64, ctypes.c_int, ctypes.c_int,
                                  pp]
    for f in ("oracle_apriori", "oracle_bruteforce", "oracle_tidlist"):
        getattr(L, f).argtypes = [p, u64, u32, ctypes.c_double, pp]
    L.oracle_item_counts.argtypes = [p, u64, u32, p]
    L.oracle_count_block.argtypes = [p, u64, u32, p, u64, u64, u64, p]
    L.oracle_result_size.restype = u64
    L.oracle_result_size.argtypes = [p]
    L.oracle_result_words.restype = u32
    L.oracle_result_words.argtypes = [p]
    L.oracle_result_masks.restype = p
    L.oracle_result_masks.argtypes = [p]
    L.oracle_result_counts.restype = p
    L.oracle_result_counts.argtypes = [p]
    L.oracle_result_stats.argtypes = [p, ctypes.POINTER(_Stats)]
    L.oracle_result_trace_len.restype = u64
    L.oracle_result_trace_len.argtypes = [p]
    L.oracle_result_trace.restype = ctypes.POINTER(_Stop)
    L.oracle_result_trace.argtypes = [p]
    L.oracle_result_free.argtypes = [p]
    L.oracle_result_free.restype = None
    L.oracle_rules.argtypes = [p, p, u64, u32, ctypes.c_double, pp]
    L.oracle_rules_size.restype = u64
    L.oracle_rules_size.argtypes = [p]
    for f in ("oracle_rules_itemset", "oracle_rules_code", "oracle_rules_supp_x"):
        getattr(L, f).restype = p
        getattr(L, f).argtypes = [p]
    L.oracle_rules_free.argtypes = [p]
    L.oracle_rules_free.restype = None
    _lib = L
    return L


@dataclass
class Result:
    masks: np.ndarray          # uint64[q, W], canonical order
    counts: np.ndarray         # uint32[q]
    stats: dict = field(default_factory=dict)
    trace: np.ndarray | None = None  # uint64[stops, 7] in TRACE_FIELDS order


def _rows(rows) -> np.ndarray:
    r = np.ascontiguousarray(rows, dtype=np.uint64)
    if r.ndim != 2:
        raise ValueError("rows must be uint64[n, W]")
    return r


def _collect(L, h, where) -> Result:
    q = L.oracle_result_size(h)
    W = L.oracle_result_words(h)
    if q:
        masks = np.ctypeslib.as_array(ctypes.cast(L.oracle_result_masks(h),
                                                  ctypes.POINTER(ctypes.c_uint64)),
                                      shape=(q * W,)).reshape(q, W).copy()
        counts = np.ctypeslib.as_array(ctypes.cast(L.oracle_result_counts(h),
                                                   ctypes.POINTER(ctypes.c_uint32)),
                                       shape=(q,)).copy()
    else:
        masks = np.zeros((0, W), np.uint64)
        counts = np.zeros(0, np.uint32)
    st = _Stats()
    L.oracle_result_stats(h, ctypes.byref(st))
    stats = {k: int(getattr(st, k)) for k, _ in _Stats._fields_}
    nt = L.oracle_result_trace_len(h)
    tr = None
    if nt:
        tp = L.oracle_result_trace(h)
        tr = np.array([[getattr(tp[i], f) for f in TRACE_FIELDS] for i in range(nt)],
                      dtype=np.uint64)
    L.oracle_result_free(h)
    return Result(masks, counts, stats, tr)


def tau(minsup: float, n: int) -> int:
    L = _load()
    out = ctypes.c_uint64()
    rc = L.oracle_tau(float(minsup), int(n), ctypes.byref(out))
    if rc:
        raise OracleError(rc, "oracle_tau")
    return int(out.value)


def dic(rows, m: int, minsup: float, M: int, candgen_mode: int = 0, init_mode: int = 0) -> Result:
    """Frequent itemsets by the oracle's serial ParallelDIC (Algorithm 2);
    init_mode 1 starts from classic DIC's all-1-itemset Dashed Circle
    (Algorithm 1) instead of FirstPass."""
    L = _load()
    r = _rows(rows)
    h = ctypes.c_void_p()
    rc = L.oracle_dic_init(r.ctypes.data, r.shape[0], int(m), float(minsup), int(M),
                           int(candgen_mode), int(init_mode), ctypes.byref(h))
    if rc:
        raise OracleError(rc, "oracle_dic")
    return _collect(L, h, "dic")


def _simple(fn, rows, m, minsup) -> Result:
    L = _load()
    r = _rows(rows)
    h = ctypes.c_void_p()
    rc = getattr(L, fn)(r.ctypes.data, r.shape[0], int(m), float(minsup), ctypes.byref(h))
    if rc:
        raise OracleError(rc, fn)
    return _collect(L, h, fn)


def apriori(rows, m, minsup) -> Result:
    return _simple("oracle_apriori", rows, m, minsup)


def bruteforce(rows, m, minsup) -> Result:
    return _simple("oracle_bruteforce", rows, m, minsup)


def tidlist(rows, m, minsup) -> Result:
    return _simple("oracle_tidlist", rows, m, minsup)


def item_counts(rows, m) -> np.ndarray:
    L = _load()
    r = _rows(rows)
    out = np.zeros(m, np.uint32)
    rc = L.oracle_item_counts(r.ctypes.data, r.shape[0], int(m), out.ctypes.data)
    if rc:
        raise OracleError(rc, "oracle_item_counts")
    return out


def count_block(rows, m, masks, first: int = 0, last: int | None = None) -> np.ndarray:
    """Rows of [first, last) containing each itemset (masks uint64[q, W])."""
    L = _load()
    r = _rows(rows)
    mk = np.ascontiguousarray(masks, dtype=np.uint64).reshape(-1, r.shape[1])
    last = r.shape[0] if last is None else last
    out = np.zeros(mk.shape[0], np.uint32)
    rc = L.oracle_count_block(r.ctypes.data, r.shape[0], int(m), mk.ctypes.data, mk.shape[0],
                              int(first), int(last), out.ctypes.data)
    if rc:
        raise OracleError(rc, "oracle_count_block")
    return out


@dataclass
class Rules:
    """Association rules X => I \\ X: itemset[r] indexes I in the input,
    code[r] selects X's items among I's ascending items, supp_x[r] = supp(X)."""
    itemset: np.ndarray  # uint32[R]
    code: np.ndarray     # uint32[R]
    supp_x: np.ndarray   # uint32[R]


def rules(masks, counts, minconf: float) -> Rules:
    """All rules of confidence >= minconf from frequent itemsets (see the C header)."""
    L = _load()
    mk = np.ascontiguousarray(masks, dtype=np.uint64)
    if mk.ndim != 2:
        raise ValueError("masks must be uint64[q, W]")
    ct = np.ascontiguousarray(counts, dtype=np.uint32)
    h = ctypes.c_void_p()
    rc = L.oracle_rules(mk.ctypes.data, ct.ctypes.data, mk.shape[0], mk.shape[1],
                        float(minconf), ctypes.byref(h))
    if rc:
        raise OracleError(rc, "oracle_rules")
    R = L.oracle_rules_size(h)

    def arr(fn):
        if not R:
            return np.zeros(0, np.uint32)
        return np.ctypeslib.as_array(ctypes.cast(fn(h), ctypes.POINTER(ctypes.c_uint32)),
                                     shape=(R,)).copy()
    out = Rules(arr(L.oracle_rules_itemset), arr(L.oracle_rules_code), arr(L.oracle_rules_supp_x))
    L.oracle_rules_free(h)
    return out
