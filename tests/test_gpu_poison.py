"""No read of memory a run has not written: every job buffer filled with a
byte pattern on allocation (option "poison") must not change any result.

Job buffers come from a cache of freed blocks, so without the fill a read
before write would see whatever an earlier job left there, and the result
would depend on what ran before (which databases share a batch, whether a
job restarted).  Each mine, batch and restart below is run with two fill
patterns and without, and all must equal each other and the oracle."""
import numpy as np
import pytest

import synth
from helpers import pack

pytestmark = pytest.mark.gpu

PATTERNS = (0xA5, 0x5A, 0xFF)


@pytest.fixture(scope="module")
def dic():
    import paper_1812_10959_amd as d
    yield d
    d.dic_set_option("poison", 0)


def _same(a, b):
    return (np.array_equal(a.masks, b.masks) and np.array_equal(a.counts, b.counts)
            and np.array_equal(a.trace, b.trace) and a.stats["stops"] == b.stats["stops"])


def _oracle_equal(r, ref):
    return (np.array_equal(r.masks, ref.masks) and np.array_equal(r.counts, ref.counts)
            and np.array_equal(r.trace.astype(np.uint64), ref.trace))


def _under(dic, byte, fn):
    dic.dic_set_option("poison", byte)
    try:
        return fn()
    finally:
        dic.dic_set_option("poison", 0)


@pytest.mark.parametrize("layout", [1, 0])
def test_single_mines_ignore_fill(dic, orc, layout):
    c = synth.config(1)
    ref = orc.dic(c["rows"], c["m"], c["minsup"], c["M"])
    db = dic.dic_load_db(c["rows"], c["m"])
    dic.dic_set_option("layout", layout)
    try:
        base = dic.dic_mine(db, c["minsup"], c["M"])
        for b in PATTERNS:
            r = _under(dic, b, lambda: dic.dic_mine(db, c["minsup"], c["M"]))
            assert _same(r, base), hex(b)
    finally:
        dic.dic_set_option("layout", 1)
    assert _oracle_equal(base, ref)


def test_batch_ignores_fill(dic):
    spec = synth.batch_config(40, seed=synth.CONFIG_SEED_BASE + 9)
    dbs = [dic.dic_load_db(d["rows"], d["m"]) for d in spec]
    ms, Ms = [d["minsup"] for d in spec], [d["M"] for d in spec]
    base = dic.dic_batch(dbs, ms, Ms)
    for b in PATTERNS:
        got = _under(dic, b, lambda: dic.dic_batch(dbs, ms, Ms))
        bad = [i for i, (x, y) in enumerate(zip(got, base)) if not _same(x, y)]
        assert not bad, (hex(b), bad[:5])
    # solo runs after the batches reuse their freed blocks
    for i in (0, 7, 39):
        assert _same(_under(dic, 0xA5, lambda: dic.dic_mine(dbs[i], ms[i], Ms[i])), base[i])


def test_restart_ignores_fill(dic, orc):
    """The pool overflows (all 65,535 itemsets of 16 items are frequent) and
    the run restarts in a new, larger pool."""
    rows = pack([list(range(16))] * 5, 16)
    db = dic.dic_load_db(rows, 16)
    ref = orc.dic(rows, 16, 0.5, 2)
    for b in (0,) + PATTERNS:
        r = _under(dic, b, lambda: dic.dic_mine(db, 0.5, 2))
        assert r.stats["restarts"] >= 1
        assert _oracle_equal(r, ref), hex(b)


def test_poison_option_is_checked(dic):
    for bad in (-1, 256):
        with pytest.raises(dic.DicError):
            dic.dic_set_option("poison", bad)
