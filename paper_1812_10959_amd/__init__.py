"""Python binding of libdic: Dynamic Itemset Counting on one MI355X (gfx950).

Thin ctypes marshalling over the C ABI of ``include/dic.h``; the functions
carry the C names (``dic_load_db``, ``dic_mine``, ``dic_batch``,
``dic_serve_*`` ...).  Every step of the mining runs in the library's HIP
kernels; there is no Python or CPU fallback, and importing this package
fails loudly when ``libdic.so`` has not been built
(``python paper_1812_10959_amd/build.py``).

PyTorch is optional plumbing: ``use_torch()`` routes the library's device
allocations through torch's caching allocator (blocks tied to torch's
current stream, on which database loads and rule generation also run; the
mining itself runs on the library's private engine streams and is complete
when a call returns), and ``dic_load_db`` accepts a CUDA/HIP tensor of
uint64 (or int64) rows already on the device.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdic.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_1812_10959_amd/build.py`")
# PyTorch ships its own HIP runtime.  Two HIP runtimes in one process cannot
# both open the GPU, so when torch is installed it is loaded first: the
# library's libamdhip64.so.7 dependency then binds to torch's copy (same
# soname) and both share one runtime, one device context and its streams.
try:
    import torch  # noqa: F401
except ImportError:
    torch = None
_lib = ctypes.CDLL(LIB_PATH)

DIC_OK = 0
DIC_E_INVAL = -1
DIC_E_NOMEM = -2
DIC_E_CAPACITY = -3
DIC_E_BUSY = -4
DIC_E_PENDING = -5
DIC_E_DEVICE = -6
DIC_E_TIMEOUT = -7
DIC_E_NOTFOUND = -8
_NAMES = {v: k for k, v in dict(globals()).items() if k.startswith("DIC_E_") or k == "DIC_OK"}

ABI_FUNCTIONS = (
    "dic_load_db", "dic_load_db_device", "dic_load_db_lists", "dic_db_rows", "dic_db_items",
    "dic_free_db", "dic_mine", "dic_mine_noalloc", "dic_batch", "dic_result_size", "dic_result_words",
    "dic_result_masks", "dic_result_counts", "dic_result_stats", "dic_result_trace",
    "dic_result_free", "dic_serve_create", "dic_serve_submit", "dic_serve_poll",
    "dic_serve_wait", "dic_serve_stats", "dic_serve_usage", "dic_serve_destroy", "dic_set_allocator",
    "dic_set_option", "dic_last_error", "dic_rules", "dic_rules_from_arrays", "dic_rules_size",
    "dic_rules_words", "dic_rules_itemset", "dic_rules_code", "dic_rules_supp_x",
    "dic_rules_antecedent", "dic_rules_consequent", "dic_rules_stats_of", "dic_rules_free",
)


class DicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class dic_stop_trace(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint32) for f in (
        "stop", "rows", "live", "promoted", "pruned", "generated", "solidified", "words", "items",
        "launch_ns")]


class dic_stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in (
        "tau", "block", "stop_max", "stops", "tests", "peak_live", "n_frequent", "k_max",
        "known", "restarts")] + [("mine_ms", ctypes.c_double), ("count_ms", ctypes.c_double),
                                 ("count_launches", ctypes.c_uint64),
                                 ("first_pass_ms", ctypes.c_double)]


class dic_rules_stats(ctypes.Structure):
    _fields_ = [("itemsets", ctypes.c_uint64), ("splits", ctypes.c_uint64),
                ("rules", ctypes.c_uint64), ("kernel_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double)]


class dic_serve_opts(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


TRACE_FIELDS = ("stop", "rows", "live", "promoted", "pruned", "generated", "solidified")

_p = ctypes.c_void_p
_pp = ctypes.POINTER(ctypes.c_void_p)
_u64, _u32, _i64 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64
_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_sig = {
    "dic_load_db": ([_p, _u64, _u32, _pp], ctypes.c_int),
    "dic_load_db_device": ([_p, _u64, _u32, _pp], ctypes.c_int),
    "dic_load_db_lists": ([_p, _p, _u64, _u32, _pp], ctypes.c_int),
    "dic_db_rows": ([_p], _u64),
    "dic_db_items": ([_p], _u32),
    "dic_free_db": ([_p], ctypes.c_int),
    "dic_mine": ([_p, ctypes.c_double, _u64, _pp], ctypes.c_int),
    "dic_mine_noalloc": ([_p, ctypes.c_double, _u64, _p, _p, _u64, ctypes.POINTER(_u64),
                          ctypes.POINTER(dic_stats)], ctypes.c_int),
    "dic_batch": ([_p, _p, _p, _u32, _p, _p], ctypes.c_int),
    "dic_result_size": ([_p], _u64),
    "dic_result_words": ([_p], _u32),
    "dic_result_masks": ([_p], _p),
    "dic_result_counts": ([_p], _p),
    "dic_result_stats": ([_p, ctypes.POINTER(dic_stats)], ctypes.c_int),
    "dic_result_trace": ([_p, ctypes.POINTER(_u64)], ctypes.POINTER(dic_stop_trace)),
    "dic_result_free": ([_p], None),
    "dic_serve_create": ([_u64, ctypes.POINTER(dic_serve_opts), _pp], ctypes.c_int),
    "dic_serve_submit": ([_p, _p, ctypes.c_double, _u64, ctypes.POINTER(_u64)], ctypes.c_int),
    "dic_serve_poll": ([_p, _u64, _pp], ctypes.c_int),
    "dic_serve_wait": ([_p, _u64, _i64, _pp], ctypes.c_int),
    "dic_serve_stats": ([_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                         ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "dic_serve_usage": ([_p, ctypes.POINTER(_u64), ctypes.POINTER(_u64), ctypes.POINTER(_u64)],
                        ctypes.c_int),
    "dic_serve_destroy": ([_p], ctypes.c_int),
    "dic_set_allocator": ([_ALLOC_T, _FREE_T, _p], ctypes.c_int),
    "dic_set_option": ([ctypes.c_char_p, _i64], ctypes.c_int),
    "dic_last_error": ([], ctypes.c_char_p),
    "dic_rules": ([_p, ctypes.c_double, _pp], ctypes.c_int),
    "dic_rules_from_arrays": ([_p, _p, _u64, _u32, ctypes.c_double, _pp], ctypes.c_int),
    "dic_rules_size": ([_p], _u64),
    "dic_rules_words": ([_p], _u32),
    "dic_rules_itemset": ([_p], _p),
    "dic_rules_code": ([_p], _p),
    "dic_rules_supp_x": ([_p], _p),
    "dic_rules_antecedent": ([_p], _p),
    "dic_rules_consequent": ([_p], _p),
    "dic_rules_stats_of": ([_p, ctypes.POINTER(dic_rules_stats)], ctypes.c_int),
    "dic_rules_free": ([_p], None),
}
for _name, (_args, _res) in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def dic_last_error() -> str:
    return (_lib.dic_last_error() or b"").decode()


def _check(rc: int, where: str) -> None:
    if rc != DIC_OK:
        raise DicError(rc, f"{where}: {dic_last_error()}")


# --------------------------------------------------------------------------- databases

class Db:
    """An owned database handle (freed by dic_free_db or garbage collection)."""

    def __init__(self, handle: int):
        self.handle = handle

    @property
    def n(self) -> int:
        return int(_lib.dic_db_rows(self.handle))

    @property
    def m(self) -> int:
        return int(_lib.dic_db_items(self.handle))

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                _lib.dic_free_db(self.handle)
            except Exception:
                pass
            self.handle = None


def _is_torch_device_tensor(x) -> bool:
    try:
        import torch
    except ImportError:
        return False
    return isinstance(x, torch.Tensor) and x.is_cuda


def dic_load_db(rows, m: int) -> Db:
    """Copy rows (uint64[n, W], W = ceil(m/64)) to the device.  ``rows`` may be
    a host array or a device tensor (copied device to device)."""
    h = ctypes.c_void_p()
    if _is_torch_device_tensor(rows):
        import torch
        if rows.dtype not in (torch.int64, torch.uint64) or rows.dim() != 2:
            raise ValueError("device rows must be a 2-D int64/uint64 tensor")
        t = rows.contiguous()
        torch.cuda.synchronize(t.device)
        _check(_lib.dic_load_db_device(t.data_ptr(), t.shape[0], int(m), ctypes.byref(h)),
               "dic_load_db_device")
        return Db(h.value)
    r = np.ascontiguousarray(rows, dtype=np.uint64)
    if r.ndim != 2 or r.shape[1] != (int(m) + 63) // 64:
        raise ValueError("rows must be uint64[n, ceil(m/64)]")
    _check(_lib.dic_load_db(r.ctypes.data, r.shape[0], int(m), ctypes.byref(h)), "dic_load_db")
    return Db(h.value)


def dic_load_db_lists(items, offsets, m: int) -> Db:
    """CSR item lists: transaction t holds items[offsets[t]:offsets[t+1]]."""
    it = np.ascontiguousarray(items, dtype=np.uint32)
    of = np.ascontiguousarray(offsets, dtype=np.uint64)
    h = ctypes.c_void_p()
    _check(_lib.dic_load_db_lists(it.ctypes.data if it.size else None, of.ctypes.data,
                                  of.size - 1, int(m), ctypes.byref(h)), "dic_load_db_lists")
    return Db(h.value)


def dic_free_db(db: Db) -> None:
    if db.handle:
        _check(_lib.dic_free_db(db.handle), "dic_free_db")
        db.handle = None


# --------------------------------------------------------------------------- results

@dataclass
class Result:
    masks: np.ndarray              # uint64[|L|, W], canonical order
    counts: np.ndarray             # uint32[|L|]
    stats: dict = field(default_factory=dict)
    trace: np.ndarray | None = None  # uint32[stops, 7] in TRACE_FIELDS order
    words: np.ndarray | None = None  # uint32[stops]: nonzero 32-bit words of the live masks
    items: np.ndarray | None = None  # uint32[stops]: items over the live candidates
    launch_ns: np.ndarray | None = None  # uint32[stops]: launch time (profile option)


def _take_result(h: int) -> Result:
    """Copy a C result into numpy arrays and free it."""
    try:
        q = int(_lib.dic_result_size(h))
        W = int(_lib.dic_result_words(h))
        if q:
            masks = np.ctypeslib.as_array(
                ctypes.cast(_lib.dic_result_masks(h), ctypes.POINTER(ctypes.c_uint64)),
                shape=(q * W,)).reshape(q, W).copy()
            counts = np.ctypeslib.as_array(
                ctypes.cast(_lib.dic_result_counts(h), ctypes.POINTER(ctypes.c_uint32)),
                shape=(q,)).copy()
        else:
            masks = np.zeros((0, W), np.uint64)
            counts = np.zeros(0, np.uint32)
        st = dic_stats()
        _check(_lib.dic_result_stats(h, ctypes.byref(st)), "dic_result_stats")
        stats = {f: (float(getattr(st, f)) if f.endswith("_ms") else int(getattr(st, f)))
                 for f, _ in dic_stats._fields_}
        ns = _u64()
        tp = _lib.dic_result_trace(h, ctypes.byref(ns))
        trace = words = items = launch = None
        if ns.value:
            raw = np.ctypeslib.as_array(ctypes.cast(tp, ctypes.POINTER(ctypes.c_uint32)),
                                        shape=(ns.value * 10,)).reshape(ns.value, 10)
            trace = raw[:, :7].copy()
            words = raw[:, 7].copy()
            items = raw[:, 8].copy()
            launch = raw[:, 9].copy()
        return Result(masks, counts, stats, trace, words, items, launch)
    finally:
        _lib.dic_result_free(h)


def dic_mine(db: Db, minsup: float, M: int) -> Result:
    """Every itemset with support >= tau and its exact count (canonical order)."""
    h = ctypes.c_void_p()
    _check(_lib.dic_mine(db.handle, float(minsup), int(M), ctypes.byref(h)), "dic_mine")
    return _take_result(h.value)


def dic_mine_noalloc(db: Db, minsup: float, M: int, capacity: int) -> Result:
    """dic_mine_noalloc into output arrays of ``capacity`` itemsets allocated
    here (the library itself allocates nothing for the call).  No per-stop
    trace.  Raises DicError (DIC_E_CAPACITY) when |L| exceeds capacity."""
    W = (db.m + 63) // 64
    masks = np.zeros((max(int(capacity), 1), W), np.uint64)
    counts = np.zeros(max(int(capacity), 1), np.uint32)
    size = _u64()
    st = dic_stats()
    _check(_lib.dic_mine_noalloc(db.handle, float(minsup), int(M), masks.ctypes.data,
                                 counts.ctypes.data, int(capacity), ctypes.byref(size),
                                 ctypes.byref(st)), "dic_mine_noalloc")
    q = int(size.value)
    stats = {f: (float(getattr(st, f)) if f.endswith("_ms") else int(getattr(st, f)))
             for f, _ in dic_stats._fields_}
    return Result(masks[:q].copy(), counts[:q].copy(), stats)


def dic_batch(dbs, minsups, Ms, raise_on_error: bool = True):
    """Mine many databases together; returns a list of Result (or DicError
    objects when ``raise_on_error`` is False)."""
    n = len(dbs)
    hs = (ctypes.c_void_p * n)(*[d.handle for d in dbs])
    ms = (ctypes.c_double * n)(*[float(x) for x in minsups])
    Mv = (ctypes.c_uint64 * n)(*[int(x) for x in Ms])
    outs = (ctypes.c_void_p * n)()
    status = (ctypes.c_int * n)()
    rc = _lib.dic_batch(hs, ms, Mv, n, outs, status)
    err = dic_last_error()
    res = []
    for i in range(n):
        if outs[i]:
            res.append(_take_result(outs[i]))
        else:
            res.append(DicError(status[i] or rc, err))
    if raise_on_error and rc != DIC_OK:
        raise DicError(rc, f"dic_batch: {err}")
    return res


# --------------------------------------------------------------------------- serving

@dataclass
class Rules:
    """Association rules X => I \\ X of a result, in (itemset, subset code) order.

    itemset[r] indexes I among the result's itemsets; bit t of code[r] selects
    the t-th smallest item of I into X; supp_x[r] = supp(X), so the confidence
    is counts[itemset[r]] / supp_x[r].  antecedent / consequent are the masks
    of X and I \\ X (uint64[R, W])."""
    itemset: np.ndarray
    code: np.ndarray
    supp_x: np.ndarray
    antecedent: np.ndarray
    consequent: np.ndarray
    stats: dict = field(default_factory=dict)


def dic_rules(result: Result, minconf: float) -> Rules:
    """Rules of confidence >= minconf from a mining result, computed on the GPU."""
    masks = np.ascontiguousarray(result.masks, dtype=np.uint64)
    counts = np.ascontiguousarray(result.counts, dtype=np.uint32)
    q, W = masks.shape
    h = _p()
    _check(_lib.dic_rules_from_arrays(masks.ctypes.data if q else None,
                                      counts.ctypes.data if q else None, q, W,
                                      float(minconf), ctypes.byref(h)), "dic_rules")
    try:
        R = int(_lib.dic_rules_size(h))

        def arr(fn, ctype, shape, dtype):
            if not R:
                return np.zeros(shape, dtype)
            ptr = ctypes.cast(fn(h), ctypes.POINTER(ctype))
            return np.ctypeslib.as_array(ptr, shape=(int(np.prod(shape)),)).reshape(shape).copy()
        st = dic_rules_stats()
        _check(_lib.dic_rules_stats_of(h, ctypes.byref(st)), "dic_rules_stats_of")
        return Rules(arr(_lib.dic_rules_itemset, ctypes.c_uint32, (R,), np.uint32),
                     arr(_lib.dic_rules_code, ctypes.c_uint32, (R,), np.uint32),
                     arr(_lib.dic_rules_supp_x, ctypes.c_uint32, (R,), np.uint32),
                     arr(_lib.dic_rules_antecedent, ctypes.c_uint64, (R, W), np.uint64),
                     arr(_lib.dic_rules_consequent, ctypes.c_uint64, (R, W), np.uint64),
                     {f: getattr(st, f) for f, _ in dic_rules_stats._fields_})
    finally:
        _lib.dic_rules_free(h)


class Server:
    def __init__(self, handle: int):
        self.handle = handle
        self.dbs = {}

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                _lib.dic_serve_destroy(self.handle)
            except Exception:
                pass
            self.handle = None


def dic_serve_create(hbm_budget_bytes: int, max_active: int = 0) -> Server:
    o = dic_serve_opts(int(max_active), 0)
    h = ctypes.c_void_p()
    _check(_lib.dic_serve_create(int(hbm_budget_bytes), ctypes.byref(o), ctypes.byref(h)),
           "dic_serve_create")
    return Server(h.value)


def dic_serve_submit(srv: Server, db: Db, minsup: float, M: int) -> int:
    t = _u64()
    _check(_lib.dic_serve_submit(srv.handle, db.handle, float(minsup), int(M), ctypes.byref(t)),
           "dic_serve_submit")
    srv.dbs[t.value] = db  # keep the database alive while the request exists
    return int(t.value)


def dic_serve_poll(srv: Server, ticket: int):
    """Result when done, None while pending; raises the request's error."""
    h = ctypes.c_void_p()
    rc = _lib.dic_serve_poll(srv.handle, int(ticket), ctypes.byref(h))
    if rc == DIC_E_PENDING:
        return None
    srv.dbs.pop(ticket, None)
    _check(rc, "dic_serve_poll")
    return _take_result(h.value)


def dic_serve_wait(srv: Server, ticket: int, timeout_ms: int = -1) -> Result:
    h = ctypes.c_void_p()
    rc = _lib.dic_serve_wait(srv.handle, int(ticket), int(timeout_ms), ctypes.byref(h))
    if rc != DIC_E_TIMEOUT:
        srv.dbs.pop(ticket, None)
    _check(rc, "dic_serve_wait")
    return _take_result(h.value)


def dic_serve_stats(srv: Server):
    """(p50 ms, p99 ms, completed requests per second)."""
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(_lib.dic_serve_stats(srv.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
           "dic_serve_stats")
    return a.value, b.value, c.value


def dic_serve_usage(srv: Server):
    """(bytes charged now, most ever charged, budget)."""
    u, p, b = _u64(), _u64(), _u64()
    _check(_lib.dic_serve_usage(srv.handle, ctypes.byref(u), ctypes.byref(p), ctypes.byref(b)),
           "dic_serve_usage")
    return u.value, p.value, b.value


def dic_serve_destroy(srv: Server) -> None:
    if srv.handle:
        _check(_lib.dic_serve_destroy(srv.handle), "dic_serve_destroy")
        srv.handle = None
        srv.dbs.clear()


# --------------------------------------------------------------------------- plumbing

_keep = []


def dic_set_allocator(alloc=None, free=None, stream: int | None = None) -> None:
    """alloc(size, stream) -> int device pointer; free(ptr, stream).  None restores
    hipMalloc/hipFree."""
    a = _ALLOC_T(alloc) if alloc else _ALLOC_T()
    f = _FREE_T(free) if free else _FREE_T()
    # every pair stays alive: blocks still go back to the free function that
    # came with their allocator after it has been replaced
    _keep.extend([a, f])
    _check(_lib.dic_set_allocator(a, f, stream or None), "dic_set_allocator")


def use_torch(stream=None) -> None:
    """Route the library's device memory through torch's caching allocator,
    with blocks tied to a torch stream (default: the current stream).  Database
    loads and dic_rules run on that stream; mining runs on the library's own
    engine streams and has finished when its call returns."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()

    def _alloc(size, _stream):
        try:
            return torch.cuda.caching_allocator_alloc(int(size), stream=s)
        except Exception:
            return None

    def _free(ptr, _stream):
        torch.cuda.caching_allocator_delete(ptr)

    dic_set_allocator(_alloc, _free, s.cuda_stream)


def dic_set_option(name: str, value: int) -> None:
    _check(_lib.dic_set_option(name.encode(), int(value)), "dic_set_option")


def _apply_tuning():
    """Apply the autotuner's saved choice (tuning.json beside this file): the
    global knobs, then the per-shape cells (all others cleared)."""
    path = os.path.join(_HERE, "tuning.json")
    _lib.dic_set_option(b"cells_clear", 1)
    if os.path.exists(path):
        import json
        with open(path) as f:
            doc = json.load(f)
        for k, v in doc.get("settings", {}).items():
            _lib.dic_set_option(k.encode(), int(v))
        for key, (mode, target) in doc.get("cells", {}).items():
            _lib.dic_set_option(f"cell:{key}".encode(), int(mode) * 65536 + int(target))


_apply_tuning()

__all__ = [n for n in ABI_FUNCTIONS] + [
    "Db", "Result", "Server", "DicError", "use_torch", "TRACE_FIELDS", "LIB_PATH",
]
