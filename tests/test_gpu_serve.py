"""GPU tests of the engine's dynamic paths: continuous-batching serving,
candidate-pool overflow and restart, and count-kernel profiling."""
import itertools
import sys
import threading
import time

import numpy as np
import pytest

import synth
from helpers import as_dict, pack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dic():
    import paper_1812_10959_amd as d
    return d


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same(a, b):
    return (np.array_equal(a.masks, b.masks) and np.array_equal(a.counts, b.counts)
            and np.array_equal(a.trace, b.trace))


def _mixed_dbs(dic):
    specs = [(3000, 64, 0.15, (0.02, 0.05)), (5000, 200, 0.03, (0.005, 0.02)),
             (800, 16, 0.4, (0.1, 0.3)), (20000, 1000, 0.008, (0.006, 0.012)),
             (4000, 128, 0.1, (0.01, 0.03))]
    out = []
    for i, (n, m, d, rng) in enumerate(specs):
        rows = synth.uniform_random(n, m, d, 700 + i)
        out.append((dic.dic_load_db(rows, m), rows, m, rng))
    return out


def test_serve_results_equal_solo(dic, orc):
    """Requests submitted while others run (a Poisson-like trickle) give the
    same itemsets, counts and traces as mining each alone, and as the oracle."""
    dbs = _mixed_dbs(dic)
    rng = np.random.default_rng(5)
    reqs = []
    for k in range(40):
        j = int(rng.integers(0, len(dbs)))
        lo, hi = dbs[j][3]
        reqs.append((j, float(rng.uniform(lo, hi)), int(rng.integers(1, 3000))))
    srv = dic.dic_serve_create(64 << 30, max_active=8)
    tickets = []
    for j, ms, M in reqs:
        tickets.append(dic.dic_serve_submit(srv, dbs[j][0], ms, M))
        time.sleep(float(rng.exponential(0.002)))
    _say(f"submitted {len(tickets)}")
    served = [dic.dic_serve_wait(srv, t, 60_000) for t in tickets]
    p50, p99, rps = dic.dic_serve_stats(srv)
    assert 0 < p50 <= p99 and rps > 0
    dic.dic_serve_destroy(srv)
    for (j, ms, M), r in zip(reqs, served):
        solo = dic.dic_mine(dbs[j][0], ms, M)
        assert _same(r, solo), (j, ms, M)
    # the oracle on the narrow databases
    for (j, ms, M), r in [x for x in zip(reqs, served) if dbs[x[0][0]][2] <= 200][:8]:
        ref = orc.dic(dbs[j][1], dbs[j][2], ms, M)
        assert np.array_equal(r.masks, ref.masks) and np.array_equal(r.counts, ref.counts)
        assert np.array_equal(r.trace.astype(np.uint64), ref.trace)


def test_serve_poll_and_errors(dic):
    rows = synth.uniform_random(2000, 64, 0.2, 1)
    db = dic.dic_load_db(rows, 64)
    srv = dic.dic_serve_create(8 << 30, max_active=2)
    t = dic.dic_serve_submit(srv, db, 0.05, 100)
    # the database is referenced: freeing it is refused
    with pytest.raises(dic.DicError) as e:
        dic.dic_free_db(db)
    assert e.value.code == dic.DIC_E_BUSY
    r = None
    for _ in range(20000):
        r = dic.dic_serve_poll(srv, t)
        if r is not None:
            break
        time.sleep(0.001)
    assert r is not None and _same(r, dic.dic_mine(db, 0.05, 100))
    with pytest.raises(dic.DicError) as e:
        dic.dic_serve_poll(srv, t)  # already handed over
    assert e.value.code == dic.DIC_E_NOTFOUND
    dic.dic_serve_destroy(srv)
    # a budget smaller than one request's memory bound
    tiny = dic.dic_serve_create(1 << 20)
    with pytest.raises(dic.DicError) as e:
        dic.dic_serve_submit(tiny, db, 0.05, 100)
    assert e.value.code == dic.DIC_E_CAPACITY
    dic.dic_serve_destroy(tiny)
    dic.dic_free_db(db)  # no longer referenced


def test_serve_admission_respects_budget(dic):
    """With room for one request at a time every request still completes."""
    rows = synth.uniform_random(3000, 100, 0.1, 2)
    db = dic.dic_load_db(rows, 100)
    srv1 = dic.dic_serve_create(64 << 30)
    t = dic.dic_serve_submit(srv1, db, 0.01, 300)
    ref = dic.dic_serve_wait(srv1, t)
    dic.dic_serve_destroy(srv1)
    # the smallest power-of-two budget that admits one request
    bound = None
    for b in (1 << 24, 1 << 26, 1 << 28, 1 << 30, 1 << 32):
        s2 = dic.dic_serve_create(b)
        try:
            t = dic.dic_serve_submit(s2, db, 0.01, 300)
            bound = b
            dic.dic_serve_wait(s2, t)
            dic.dic_serve_destroy(s2)
            break
        except dic.DicError:
            dic.dic_serve_destroy(s2)
    assert bound is not None
    srv = dic.dic_serve_create(bound, max_active=4)
    ts = [dic.dic_serve_submit(srv, db, 0.01, 300) for _ in range(5)]
    for t in ts:
        assert _same(dic.dic_serve_wait(srv, t), ref)
    dic.dic_serve_destroy(srv)


def test_pool_overflow_restarts(dic, orc):
    """16 items in every row: all 65,535 itemsets are frequent, far beyond
    the first candidate pool (4 * 120 pairs + 16,384); the run restarts with
    more room and still returns the closed-form answer."""
    n, T = 6, list(range(16))
    rows = pack([T] * n, 16)
    db = dic.dic_load_db(rows, 16)
    r = dic.dic_mine(db, 0.5, 2)
    assert r.stats["restarts"] >= 1
    assert len(r.counts) == 2 ** 16 - 1 and set(r.counts.tolist()) == {n}
    ref = orc.dic(rows, 16, 0.5, 2)
    assert np.array_equal(r.masks, ref.masks) and np.array_equal(r.counts, ref.counts)
    assert np.array_equal(r.trace.astype(np.uint64), ref.trace)


def test_profile_option_times_count_kernel(dic):
    c = synth.config(1)
    db = dic.dic_load_db(c["rows"], 64)
    dic.dic_set_option("profile", 1)
    r = dic.dic_mine(db, c["minsup"], c["M"])
    dic.dic_set_option("profile", 0)
    assert r.stats["count_launches"] >= r.stats["stops"] > 0
    assert 0 < r.stats["count_ms"] < r.stats["mine_ms"]
    r2 = dic.dic_mine(db, c["minsup"], c["M"])
    assert r2.stats["count_ms"] == 0 and _same(r, r2)
    # per-stop work counters: every live candidate has at least two items, and
    # with row bitmaps at least one nonzero mask word
    assert (r.items >= 2 * r.trace[:, 2]).all()
    dic.dic_set_option("layout", 0)
    dic.dic_set_option("profile", 1)
    try:
        rr = dic.dic_mine(db, c["minsup"], c["M"])
    finally:
        dic.dic_set_option("profile", 0)
        dic.dic_set_option("layout", 1)
    assert (rr.words >= rr.trace[:, 2]).all() and _same(rr, r)
    with pytest.raises(dic.DicError):
        dic.dic_set_option("no-such-option", 1)


def test_concurrent_host_threads(dic):
    """dic_mine on different databases from several host threads at once."""
    items = []
    for i in range(4):
        rows = synth.uniform_random(4000, 96, 0.1, 900 + i)
        db = dic.dic_load_db(rows, 96)
        items.append((db, dic.dic_mine(db, 0.01, 500)))
    out = [None] * 4

    def work(i):
        out[i] = dic.dic_mine(items[i][0], 0.01, 500)

    th = [threading.Thread(target=work, args=(i,)) for i in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for i in range(4):
        assert _same(out[i], items[i][1])


def test_planning_knobs_do_not_change_results(dic, orc):
    """Every tuning knob setting gives the oracle's result (tile and wave modes,
    tile shapes, grid sizes, row-bitmap work split)."""
    rows, _ = synth.quest(6000, 200, n_patterns=150, pat_len_mean=4, txn_len_mean=9, seed=77,
                          zipf_s=1.1)
    ref = orc.dic(rows, 200, 0.006, 700)
    db = dic.dic_load_db(rows, 200)
    base = {"vt_target": 768, "vt_wave_k": 2048, "vt_tile_words": 16, "count_grid": 2048,
            "count_target": 2048}
    variants = [dict(vt_wave_k=0), dict(vt_wave_k=1 << 20), dict(vt_tile_words=1),
                dict(vt_tile_words=5), dict(vt_target=64), dict(vt_target=8192),
                dict(count_grid=64), dict(count_grid=5000)]
    # per-shape cells: all wave, all tiles at a small and a large target,
    # and a checkerboard of both
    cells = [{(b, k): (1, 0) for b in range(5) for k in range(5)},
             {(b, k): (2, 64) for b in range(5) for k in range(5)},
             {(b, k): (2, 4096) for b in range(5) for k in range(5)},
             {(b, k): ((1, 0) if (b + k) % 2 else (2, 300)) for b in range(5) for k in range(5)}]
    try:
        dic.dic_set_option("cells_clear", 1)
        for v in variants + cells:
            if v in cells:
                for k, x in base.items():
                    dic.dic_set_option(k, x)
                for (b, k), (mode, target) in v.items():
                    dic.dic_set_option(f"cell:{b}:{k}", mode * 65536 + target)
            else:
                for k, x in {**base, **v}.items():
                    dic.dic_set_option(k, x)
            g = dic.dic_mine(db, 0.006, 700)
            dic.dic_set_option("cells_clear", 1)
            assert np.array_equal(g.masks, ref.masks) and np.array_equal(g.counts, ref.counts), v
            assert np.array_equal(g.trace.astype(np.uint64), ref.trace), v
        dic.dic_set_option("layout", 0)
        for ct in (64, 100000 // 10):
            dic.dic_set_option("count_target", ct)
            g = dic.dic_mine(db, 0.006, 700)
            assert np.array_equal(g.counts, ref.counts), ct
    finally:
        dic.dic_set_option("layout", 1)
        for k, x in base.items():
            dic.dic_set_option(k, x)
        import paper_1812_10959_amd
        paper_1812_10959_amd._apply_tuning()
    with pytest.raises(dic.DicError):
        dic.dic_set_option("vt_tile_words", 17)
    for bad in (("cell:5:0", 65536), ("cell:0:5", 65536), ("cell:0:0", 3 * 65536),
                ("cell:0:0", 2 * 65536 + 10), ("cell:0", 65536), ("cell:0:0:1", 65536)):
        with pytest.raises(dic.DicError):
            dic.dic_set_option(*bad)
