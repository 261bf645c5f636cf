"""GPU association rules (dic_rules) against the oracle's rules.

Both sides start from a mining result: the GPU mines and derives rules on the
device, the oracle derives rules from its own mining result (or from the
golden itemsets the oracle wrote).  Rules are compared element by element in
(itemset, subset code) order; supports are exact and both sides take the
keep decision with the same double-precision expression.
"""
import gzip
import json
import os

import numpy as np
import pytest

import synth
from helpers import items_of, pack

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _say(*a):
    print(*a, flush=True)


def _code_masks(masks, itemset, code):
    """Antecedent / consequent masks from (itemset, code), computed independently."""
    W = masks.shape[1]
    ante = np.zeros((len(itemset), W), np.uint64)
    cons = np.zeros((len(itemset), W), np.uint64)
    for r, (i, c) in enumerate(zip(itemset, code)):
        I = items_of(masks[i])
        for t, p in enumerate(I):
            tgt = ante if (int(c) >> t) & 1 else cons
            tgt[r, p >> 6] |= np.uint64(1) << np.uint64(p & 63)
    return ante, cons


def _assert_same(g, ref, masks, label):
    assert len(g.itemset) == len(ref.itemset), (label, len(g.itemset), len(ref.itemset))
    assert np.array_equal(g.itemset, ref.itemset), label
    assert np.array_equal(g.code, ref.code), label
    assert np.array_equal(g.supp_x, ref.supp_x), label
    if len(g.itemset) <= 200000:
        ante, cons = _code_masks(masks, g.itemset, g.code)
        assert np.array_equal(g.antecedent, ante), label
        assert np.array_equal(g.consequent, cons), label


def test_hand_example(orc):
    import paper_1812_10959_amd as dic
    g = json.load(open(os.path.join(GOLDEN, "rules_hand_example.json")))
    names = g["items"]
    idx = {c: i for i, c in enumerate(names)}
    rows = pack([[idx[c] for c in t] for t in g["transactions"]], len(names))
    res = dic.dic_mine(dic.dic_load_db(rows, len(names)), g["minsup"], 1)
    for case in g["cases"]:
        R = dic.dic_rules(res, case["minconf"])
        got = set()
        for i, c in zip(R.itemset, R.code):
            I = items_of(res.masks[i])
            X = "".join(names[p] for t, p in enumerate(I) if (int(c) >> t) & 1)
            Y = "".join(names[p] for t, p in enumerate(I) if not (int(c) >> t) & 1)
            got.add((X, Y))
        assert got == {tuple(r) for r in case["rules"]}, case["note"]


@pytest.mark.parametrize("seed", range(5))
def test_random_databases(orc, seed):
    import paper_1812_10959_amd as dic
    rng = np.random.default_rng(7100 + seed)
    n, m = int(rng.integers(200, 3000)), int(rng.choice([12, 40, 70, 130]))
    rows = synth.uniform_random(n, m, float(rng.uniform(0.1, 0.3)), seed=7100 + seed)
    minsup = float(rng.uniform(0.02, 0.08))
    M = int(rng.integers(1, n + 1))
    g_res = dic.dic_mine(dic.dic_load_db(rows, m), minsup, M)
    o_res = orc.dic(rows, m, minsup, M)
    assert np.array_equal(g_res.masks, o_res.masks)
    for minconf in (0.0, 0.25, 0.6, 0.9, 1.0):
        _say(f"seed {seed} n={n} m={m} |L|={len(o_res.counts)} minconf={minconf}")
        g = dic.dic_rules(g_res, minconf)
        ref = orc.rules(o_res.masks, o_res.counts, minconf)
        _assert_same(g, ref, o_res.masks, (seed, minconf))
        assert g.stats["rules"] == len(ref.itemset)


def test_config1_full_size(orc):
    import paper_1812_10959_amd as dic
    c = synth.config(1)
    g_res = dic.dic_mine(dic.dic_load_db(c["rows"], c["m"]), c["minsup"], c["M"])
    o_res = orc.dic(c["rows"], c["m"], c["minsup"], c["M"])
    for minconf in (0.3, 0.7):
        g = dic.dic_rules(g_res, minconf)
        ref = orc.rules(o_res.masks, o_res.counts, minconf)
        _say(f"config 1: |L|={len(o_res.counts)} rules={len(ref.itemset)} at {minconf}")
        _assert_same(g, ref, o_res.masks, minconf)


def _golden_itemsets(index):
    items, counts = [], []
    with gzip.open(os.path.join(GOLDEN, f"workload{index}.itemsets.txt.gz"), "rt") as f:
        for ln in f:
            a, c = ln.rstrip("\n").split("\t")
            items.append([int(x) for x in a.split(",")])
            counts.append(int(c))
    return items, np.array(counts, np.uint32)


@pytest.mark.parametrize("index", [3, 2])
def test_workload_rules(orc, index):
    """Rules of the large workloads: GPU mine + GPU rules vs oracle rules of the
    golden (oracle-written) itemsets."""
    import paper_1812_10959_amd as dic
    c = synth.config(index)
    items, counts = _golden_itemsets(index)
    W = c["rows"].shape[1]
    masks = np.zeros((len(items), W), np.uint64)
    for r, it in enumerate(items):
        for p in it:
            masks[r, p >> 6] |= np.uint64(1) << np.uint64(p & 63)
    g_res = dic.dic_mine(dic.dic_load_db(c["rows"], c["m"]), c["minsup"], c["M"])
    assert np.array_equal(g_res.masks, masks) and np.array_equal(g_res.counts, counts)
    for minconf in (0.5, 0.9):
        g = dic.dic_rules(g_res, minconf)
        ref = orc.rules(masks, counts, minconf)
        _say(f"workload {index}: splits={g.stats['splits']} rules={len(ref.itemset)} "
             f"kernel {g.stats['kernel_ms']:.3f} ms")
        _assert_same(g, ref, masks, (index, minconf))


def test_edge_cases(orc):
    import paper_1812_10959_amd as dic
    from paper_1812_10959_amd import DicError, DIC_E_INVAL
    # identical transactions: every split is a rule of confidence 1
    t = 6
    rows = pack([list(range(t))] * 9, 64)
    res = dic.dic_mine(dic.dic_load_db(rows, 64), 0.5, 4)
    assert len(res.counts) == 2 ** t - 1
    assert len(dic.dic_rules(res, 1.0).itemset) == 3 ** t - 2 ** (t + 1) + 1
    assert len(dic.dic_rules(res, 1.0000001).itemset) == 0
    # only 1-itemsets: no rules; empty result: no rules
    rows1 = pack([[0], [1], [2], [0], [1], [2]], 8)
    res1 = dic.dic_mine(dic.dic_load_db(rows1, 8), 0.3, 2)
    assert len(res1.counts) == 3 and len(dic.dic_rules(res1, 0.0).itemset) == 0
    res0 = dic.dic_mine(dic.dic_load_db(rows1, 8), 0.9, 2)
    assert len(res0.counts) == 0 and len(dic.dic_rules(res0, 0.1).itemset) == 0
    # errors: NaN, too large an itemset, not downward closed
    with pytest.raises(DicError) as e:
        dic.dic_rules(res, float("nan"))
    assert e.value.code == DIC_E_INVAL
    big = dic.Result(np.array([[(1 << 25) - 1]], np.uint64), np.array([3], np.uint32))
    with pytest.raises(DicError) as e:
        dic.dic_rules(big, 0.5)
    assert e.value.code == DIC_E_INVAL
    open_set = dic.Result(np.array([[0b1], [0b11]], np.uint64), np.array([5, 3], np.uint32))
    with pytest.raises(DicError) as e:
        dic.dic_rules(open_set, 0.5)
    assert e.value.code == DIC_E_INVAL
    # the same splits as the oracle on a result with 1 <= k <= 12 itemsets
    ref = orc.rules(res.masks, res.counts, 0.0)
    _assert_same(dic.dic_rules(res, 0.0), ref, res.masks, "identical rows")
