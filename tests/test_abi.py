"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments on the host (no GPU needed: none of these calls reach the device)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dic.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^DIC_API[^(]*?\b(dic_\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def dic():
    import paper_1812_10959_amd as d
    return d


def test_header_declares_the_boundary():
    names = _declared()
    for need in ("dic_load_db", "dic_load_db_lists", "dic_free_db", "dic_mine", "dic_batch",
                 "dic_result_size", "dic_result_masks", "dic_result_counts", "dic_result_stats",
                 "dic_result_free", "dic_serve_create", "dic_serve_submit", "dic_serve_poll",
                 "dic_serve_wait", "dic_serve_stats", "dic_serve_destroy", "dic_set_allocator",
                 "dic_last_error"):
        assert need in names


def test_library_exports_every_declared_symbol(dic):
    lib = ctypes.CDLL(dic.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing
    assert sorted(dic.ABI_FUNCTIONS) == _declared()


def test_library_is_gfx950(dic):
    # the device code object in the library targets gfx950 only
    blob = open(dic.LIB_PATH, "rb").read()
    assert b"gfx950" in blob
    for other in (b"gfx942", b"gfx90a", b"gfx1100"):
        assert other not in blob


def test_host_side_validation(dic):
    lib = dic._lib
    h = ctypes.c_void_p()
    # NULL / shape errors
    assert lib.dic_load_db(None, 10, 64, ctypes.byref(h)) == dic.DIC_E_INVAL and not h.value
    rows = np.zeros((4, 1), np.uint64)
    assert lib.dic_load_db(rows.ctypes.data, 0, 64, ctypes.byref(h)) == dic.DIC_E_INVAL
    assert lib.dic_load_db(rows.ctypes.data, 4, 0, ctypes.byref(h)) == dic.DIC_E_INVAL
    assert lib.dic_load_db(rows.ctypes.data, 4, 5000, ctypes.byref(h)) == dic.DIC_E_INVAL
    assert lib.dic_load_db(rows.ctypes.data, 2**32 - 1, 64, ctypes.byref(h)) == dic.DIC_E_INVAL
    # a padding bit (item 10 with m = 10)
    bad = np.array([[0], [1 << 10]], np.uint64)
    assert lib.dic_load_db(bad.ctypes.data, 2, 10, ctypes.byref(h)) == dic.DIC_E_INVAL
    assert "at or above m" in dic.dic_last_error()
    # lists: item out of range, decreasing offsets
    items = np.array([0, 3, 9], np.uint32)
    offs = np.array([0, 2, 3], np.uint64)
    assert lib.dic_load_db_lists(items.ctypes.data, offs.ctypes.data, 2, 9,
                                 ctypes.byref(h)) == dic.DIC_E_INVAL
    offs2 = np.array([0, 2, 1], np.uint64)
    assert lib.dic_load_db_lists(items.ctypes.data, offs2.ctypes.data, 2, 64,
                                 ctypes.byref(h)) == dic.DIC_E_INVAL
    # mining arguments
    out = ctypes.c_void_p()
    assert lib.dic_mine(None, 0.5, 10, ctypes.byref(out)) == dic.DIC_E_INVAL and not out.value
    # NULL-safe accessors and frees
    assert lib.dic_free_db(None) == dic.DIC_OK
    lib.dic_result_free(None)
    assert lib.dic_result_size(None) == 0
    assert lib.dic_db_rows(None) == 0
    # allocator hook: both functions or neither
    assert lib.dic_set_allocator(dic._ALLOC_T(lambda s, t: None), dic._FREE_T(), None) == \
        dic.DIC_E_INVAL


def test_python_wrappers_raise(dic):
    with pytest.raises(ValueError):
        dic.dic_load_db(np.zeros((3, 2), np.uint64), 64)  # W mismatch
    with pytest.raises(dic.DicError) as e:
        dic.dic_load_db(np.array([[1 << 63]], np.uint64), 63)
    assert e.value.code == dic.DIC_E_INVAL


def test_oracle_and_library_share_nothing():
    """The oracle tree and the GPU library neither include nor import each other."""
    odir = os.path.join(ROOT, "oracle")
    pdir = os.path.join(ROOT, "paper_1812_10959_amd")
    for d, forbidden in ((odir, ("paper_1812_10959_amd", "dic.h", "dic_internal")),
                         (pdir, ("oracle", "dic_oracle"))):
        for base, _, files in os.walk(d):
            for f in files:
                if f.endswith((".py", ".c", ".h", ".hip", ".cpp")):
                    txt = open(os.path.join(base, f)).read()
                    for word in forbidden:
                        assert not re.search(rf"(import|include)[^\n]*\b{word}\b", txt), (f, word)
