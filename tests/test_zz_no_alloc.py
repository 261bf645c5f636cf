"""dic_mine_noalloc (working memory from a static device array, nothing
allocated per call) gives exactly what dic_mine gives: the same itemsets in
canonical order, the same counts and the same statistics.  Two calls in a
row, the second on a smaller database, so that the second starts on the
array the first left behind; both also equal the CPU oracle."""
import ctypes
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

STAT_KEYS = ("tau", "block", "stop_max", "stops", "tests", "peak_live", "n_frequent", "k_max",
             "known")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _noalloc_abi(dic, db, minsup, M, capacity):
    """The C entry point called directly through ctypes."""
    W = (db.m + 63) // 64
    masks = np.full((max(capacity, 1), W), 0xDEADBEEF, np.uint64)
    counts = np.full(max(capacity, 1), 7, np.uint32)
    size = ctypes.c_uint64()
    st = dic.dic_stats()
    rc = dic._lib.dic_mine_noalloc(db.handle, ctypes.c_double(minsup), ctypes.c_uint64(M),
                                   masks.ctypes.data, counts.ctypes.data,
                                   ctypes.c_uint64(capacity), ctypes.byref(size),
                                   ctypes.byref(st))
    stats = {k: int(getattr(st, k)) for k in STAT_KEYS}
    return rc, int(size.value), masks, counts, stats


def _check_equal(dic, orc, rows, m, minsup, M, label):
    db = dic.dic_load_db(rows, m)
    ref = dic.dic_mine(db, minsup, M)
    q = len(ref.counts)
    _say(f"{label}: n={rows.shape[0]} m={m} |L|={q} stops={ref.stats['stops']}")
    rc, size, masks, counts, stats = _noalloc_abi(dic, db, minsup, M, q + 5)
    assert rc == dic.DIC_OK, dic.dic_last_error()
    assert size == q
    assert np.array_equal(masks[:q], ref.masks)
    assert np.array_equal(counts[:q], ref.counts)
    for k in STAT_KEYS:
        assert stats[k] == ref.stats[k], (label, k, stats[k], ref.stats[k])
    o = orc.dic(rows, m, minsup, M)
    assert np.array_equal(masks[:q], o.masks) and np.array_equal(counts[:q], o.counts)
    # an output array one itemset short: DIC_E_CAPACITY, the size reported
    if q:
        rc, size, _, _, _ = _noalloc_abi(dic, db, minsup, M, q - 1)
        assert rc == dic.DIC_E_CAPACITY and size == q
    return db


def test_noalloc_equals_dic_mine_twice_second_smaller(orc):
    import paper_1812_10959_amd as dic
    big = synth.config(1)  # n = 10,000, m = 64, minsup 2 %, M = 1,000
    _check_equal(dic, orc, big["rows"], big["m"], big["minsup"], big["M"], "first call")
    small, _ = synth.quest(2_500, 40, n_patterns=60, pat_len_mean=4, txn_len_mean=7, seed=77)
    _check_equal(dic, orc, small, 40, 0.03, 300, "second call (smaller)")


def test_noalloc_layouts_and_classic_start(orc):
    import paper_1812_10959_amd as dic
    rows, _ = synth.quest(3_000, 130, n_patterns=150, pat_len_mean=4, txn_len_mean=9, seed=5)
    try:
        for layout, init in ((0, 0), (1, 1), (1, 0)):
            dic.dic_set_option("layout", layout)
            dic.dic_set_option("init", init)
            _check_equal(dic, orc, rows, 130, 0.02, 500, f"layout {layout} init {init}")
    finally:
        dic.dic_set_option("layout", 1)
        dic.dic_set_option("init", 0)


def test_noalloc_rejects_a_mine_larger_than_its_array():
    import paper_1812_10959_amd as dic
    # every one of 1,024 items frequent: about 5 * 10^5 pair candidates, far
    # more working memory than the static array holds
    rows = np.full((64, 16), np.uint64(0xFFFFFFFFFFFFFFFF), np.uint64)
    db = dic.dic_load_db(rows, 1024)
    rc, size, _, _, _ = _noalloc_abi(dic, db, 0.5, 16, 10)
    assert rc == dic.DIC_E_CAPACITY
    assert "working memory" in dic.dic_last_error()
    # and the array still serves a normal call afterwards
    c = synth.config(1)
    db2 = dic.dic_load_db(c["rows"], c["m"])
    ref = dic.dic_mine(db2, c["minsup"], c["M"])
    rc, size, masks, counts, _ = _noalloc_abi(dic, db2, c["minsup"], c["M"], len(ref.counts))
    assert rc == dic.DIC_OK and size == len(ref.counts)
    assert np.array_equal(masks[:size], ref.masks) and np.array_equal(counts[:size], ref.counts)
