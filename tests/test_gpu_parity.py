"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Counts are integers, so the bar is bit-exact: the same itemsets in the same
canonical order, the same uint32 counts, the same threshold, stop count,
subset-test total and per-stop trace (live, promoted, pruned, generated,
solidified at every stop).
"""
import json
import os
import sys

import numpy as np
import pytest

import synth
from helpers import as_dict, is_canonical, pack

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
STAT_KEYS = ("tau", "block", "stop_max", "stops", "tests", "peak_live", "n_frequent", "k_max",
             "known")


@pytest.fixture(scope="module")
def dic():
    import paper_1812_10959_amd as d
    return d


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def assert_same(gpu, ref, label=""):
    assert gpu.masks.shape == ref.masks.shape, (label, gpu.masks.shape, ref.masks.shape)
    assert np.array_equal(gpu.masks, ref.masks), label
    assert np.array_equal(gpu.counts, ref.counts), label
    for k in STAT_KEYS:
        assert gpu.stats[k] == ref.stats[k], (label, k, gpu.stats[k], ref.stats[k])
    if ref.trace is None:
        assert gpu.trace is None or len(gpu.trace) == 0, label
    else:
        assert np.array_equal(gpu.trace.astype(np.uint64), ref.trace), label


LAYOUTS = (1, 0)  # item bitsets (default), row bitmaps


def mine_both(dic, orc, rows, m, minsup, M, label=""):
    """Mine on the GPU with both counting layouts and compare each with the oracle."""
    _say(f"case {label}: n={rows.shape[0]} m={m} minsup={minsup} M={M}")
    db = dic.dic_load_db(rows, m)
    r = orc.dic(rows, m, minsup, M)
    out = None
    for layout in LAYOUTS:
        dic.dic_set_option("layout", layout)
        try:
            g = dic.dic_mine(db, minsup, M)
        finally:
            dic.dic_set_option("layout", 1)
        assert_same(g, r, f"{label} layout={layout}")
        assert is_canonical(g.masks)
        out = out or g
    return out


def test_hand_example(dic, orc):
    gd = json.load(open(os.path.join(GOLDEN, "hand_example.json")))
    rows = pack(gd["rows"], gd["m"])
    want = {tuple(i): c for i, c in gd["frequent"]}
    for run in gd["runs"]:
        g = mine_both(dic, orc, rows, gd["m"], gd["minsup"], run["M"], f"hand M={run['M']}")
        assert as_dict(g.masks, g.counts) == want
        assert g.trace.tolist() == run["trace"]
        assert g.stats["tests"] == run["tests"]


@pytest.mark.parametrize("seed,n,m,density,minsup,Ms", [
    (1, 300, 16, 0.35, 0.05, (1, 7, 64, 300)),
    (2, 1000, 64, 0.12, 0.02, (1, 100, 333, 1000, 5000)),
    (3, 777, 65, 0.10, 0.015, (50, 129)),
    (4, 1500, 128, 0.05, 0.01, (97, 1500)),
    (5, 600, 200, 0.04, 0.008, (64, 601)),
    (6, 900, 1000, 0.008, 0.012, (100, 450)),
    (7, 2500, 1090, 0.004, 0.003, (256,)),
    (8, 64, 30, 0.6, 0.3, (1, 5, 64)),
])
def test_random_databases(dic, orc, seed, n, m, density, minsup, Ms):
    rows = synth.uniform_random(n, m, density, seed)
    for M in Ms:
        mine_both(dic, orc, rows, m, minsup, M, f"rand{seed} M={M}")


def test_quest_small(dic, orc):
    for i, (n, m, pats) in enumerate([(3000, 64, 50), (5000, 300, 200), (4000, 1000, 400)]):
        rows, _ = synth.quest(n, m, n_patterns=pats, pat_len_mean=4, txn_len_mean=9,
                              seed=100 + i, zipf_s=1.1 if m > 100 else None)
        for minsup, M in ((0.01, n // 10), (0.005, 333)):
            mine_both(dic, orc, rows, m, minsup, M, f"quest{i} ms={minsup}")


def test_many_new_candidates_at_one_stop(dic, orc):
    """Stops that create thousands of candidates at once, and long blocks.

    The candidates created at a stop are counted on the next block right
    after their creation.  From 1024 of them the item-bitset layout counts
    them on LDS tiles of the block, split in chunks over workgroups, instead
    of one wave each.  This database (Quest, 256 items, long baskets)
    creates over 4000 at its busiest stop with short blocks (even and ragged
    sizes).  With M = 16,500 the blocks alternate between 16,500 rows (258
    words, many chunks) and a ragged 3,500, and over 11,000 candidates
    created at a short block's stop are counted on a long block.
    """
    rows, _ = synth.quest(20000, 256, n_patterns=512, pat_len_mean=4, txn_len_mean=16, seed=7)
    for M in (1000, 997, 16500):
        g = mine_both(dic, orc, rows, 256, 0.01, M, f"many-new M={M}")
        gen = g.trace[:, 5].astype(np.int64)
        if M < 16500:
            assert (gen >= 1024).sum() >= 3, gen.max()
        else:
            assert gen[g.trace[:, 1] == 3500].max() >= 1024


def test_workload_one_full(dic, orc):
    c = synth.config(1)
    g = mine_both(dic, orc, c["rows"], c["m"], c["minsup"], c["M"], "config n10k m64")
    assert g.stats["n_frequent"] > 500


def test_edge_cases(dic, orc):
    # single transaction; all subsets frequent
    rows = pack([[0, 5, 63, 64, 100]], 128)
    mine_both(dic, orc, rows, 128, 1.0, 1, "single row")
    # identical rows, M not dividing n
    rows = pack([[1, 4, 5, 9, 11, 70]] * 37, 80)
    g = mine_both(dic, orc, rows, 80, 0.9, 5, "identical rows")
    assert len(g.counts) == 63 and set(g.counts.tolist()) == {37}
    # twelve items in most rows: all 4,095 subsets frequent; itemsets of 10
    # to 12 items agree on their first nine (the result sort must break ties)
    rows = pack([list(range(3, 15))] * 9 + [[0, 1, 70]], 71)
    g = mine_both(dic, orc, rows, 71, 0.5, 4, "twelve-item rows")
    assert len(g.counts) == 4095 and g.stats["k_max"] == 12
    # unreachable threshold: empty result, no stops
    rows = synth.uniform_random(50, 20, 0.9, 3)
    g = mine_both(dic, orc, rows, 20, 1.5, 7, "minsup>1")
    assert len(g.counts) == 0 and g.stats["stops"] == 0
    # fewer than two frequent items: no candidates at all
    rows = pack([[0], [0], [1], [2]], 8)
    g = mine_both(dic, orc, rows, 8, 0.5, 2, "one frequent item")
    assert g.stats["stops"] == 0
    # empty transactions are legal
    rows = pack([[], [1, 2], [], [1, 2, 3], []], 4)
    mine_both(dic, orc, rows, 4, 0.2, 2, "empty rows")
    # M larger than n, tau = 1 (everything present once is frequent)
    rows = synth.uniform_random(40, 12, 0.3, 9)
    mine_both(dic, orc, rows, 12, 1e-6, 1000, "tau=1")
    # m not a multiple of 64 and exactly 64
    for m in (1, 2, 63, 64):
        rows = synth.uniform_random(200, m, 0.5, m)
        mine_both(dic, orc, rows, m, 0.2, 17, f"m={m}")


def test_itemsets_of_every_record_form(dic, orc):
    """A live record carries up to 8 items; lists of 9 to 16 items are read
    from the pool and larger itemsets are counted from their masks.  Every
    subset of a 17-item pattern is frequent here (131,071 itemsets, sizes 1
    to 17), so all three forms are counted and pruned at many stops."""
    rows = pack([list(range(17))] * 4 + [[0, 1], [2, 3, 4], [17, 18]], 20)
    g = mine_both(dic, orc, rows, 20, 0.5, 2, "17-item pattern")
    assert g.stats["k_max"] == 17 and len(g.counts) == 131071
    rows = pack([list(range(3, 23))] * 3 + [[1, 2]] * 2, 30)
    g = mine_both(dic, orc, rows, 30, 0.6, 1, "20-item pattern, M=1")
    assert g.stats["k_max"] == 20


def test_load_paths_agree(dic, orc):
    rows = synth.uniform_random(500, 150, 0.07, 21)
    items, offs = synth.bitmap_to_csr(rows, 150)
    a = dic.dic_mine(dic.dic_load_db(rows, 150), 0.02, 64)
    b = dic.dic_mine(dic.dic_load_db_lists(items, offs, 150), 0.02, 64)
    assert np.array_equal(a.masks, b.masks) and np.array_equal(a.counts, b.counts)
    import torch
    t = torch.from_numpy(rows.view(np.int64)).cuda()
    c = dic.dic_mine(dic.dic_load_db(t, 150), 0.02, 64)
    assert np.array_equal(a.masks, c.masks) and np.array_equal(a.counts, c.counts)
    r = orc.dic(rows, 150, 0.02, 64)
    assert_same(a, r)


def test_device_padding_check(dic):
    import torch
    bad = torch.tensor([[0], [1 << 20]], dtype=torch.int64, device="cuda")
    with pytest.raises(dic.DicError) as e:
        dic.dic_load_db(bad, 20)
    assert e.value.code == dic.DIC_E_INVAL


def test_batch_mixed_layouts(dic, orc):
    """Jobs of both layouts in one engine give the oracle's results."""
    rows_a = synth.uniform_random(800, 100, 0.08, 41)
    rows_b = synth.uniform_random(600, 64, 0.15, 42)
    a, b = dic.dic_load_db(rows_a, 100), dic.dic_load_db(rows_b, 64)
    dic.dic_set_option("layout", 0)
    try:
        ra = dic.dic_batch([a, b], [0.02, 0.03], [77, 600])
    finally:
        dic.dic_set_option("layout", 1)
    rb = dic.dic_batch([a, b], [0.02, 0.03], [77, 600])
    for x, y, rows, m, ms, M in ((ra[0], rb[0], rows_a, 100, 0.02, 77),
                                 (ra[1], rb[1], rows_b, 64, 0.03, 600)):
        ref = orc.dic(rows, m, ms, M)
        assert_same(x, ref)
        assert_same(y, ref)


def test_batch_equals_solo(dic, orc):
    specs = [(400, 64, 0.2, 0.03, 40), (1200, 130, 0.05, 0.01, 100), (90, 16, 0.5, 0.2, 9),
             (2000, 1000, 0.005, 0.004, 250), (50, 8, 0.9, 2.0, 5), (700, 256, 0.03, 0.01, 35)]
    dbs, rows_l = [], []
    for i, (n, m, d, ms, M) in enumerate(specs):
        rows = synth.uniform_random(n, m, d, 300 + i)
        rows_l.append(rows)
        dbs.append(dic.dic_load_db(rows, m))
    res = dic.dic_batch(dbs, [s[3] for s in specs], [s[4] for s in specs])
    for i, (n, m, d, ms, M) in enumerate(specs):
        solo = dic.dic_mine(dbs[i], ms, M)
        assert_same(res[i], solo, f"batch elem {i}")
        assert_same(res[i], orc.dic(rows_l[i], m, ms, M), f"batch elem {i} vs oracle")


def test_repeat_calls_deep_itemsets(dic, orc):
    """Deep candidates (subset lookups through the hash table) mined again and
    again on recycled device memory: every run equals the oracle."""
    c = synth.config(3, n=20_000)
    ref = orc.dic(c["rows"], c["m"], c["minsup"], 2_000)
    assert ref.stats["k_max"] >= 6
    db = dic.dic_load_db(c["rows"], c["m"])
    for rep in range(6):
        g = dic.dic_mine(db, c["minsup"], 2_000)
        assert_same(g, ref, f"repeat {rep}")
    rows, _ = synth.quest(5000, 300, n_patterns=200, pat_len_mean=4, txn_len_mean=9, seed=101,
                          zipf_s=1.1)
    ref = orc.dic(rows, 300, 0.005, 333)
    db = dic.dic_load_db(rows, 300)
    for rep in range(4):
        assert_same(dic.dic_mine(db, 0.005, 333), ref, f"quest repeat {rep}")


def test_repeat_calls_identical(dic):
    c = synth.config(1)
    db = dic.dic_load_db(c["rows"], 64)
    a = dic.dic_mine(db, 0.02, 1000)
    for _ in range(3):
        b = dic.dic_mine(db, 0.02, 1000)
        assert np.array_equal(a.masks, b.masks) and np.array_equal(a.counts, b.counts)
        assert np.array_equal(a.trace, b.trace)
