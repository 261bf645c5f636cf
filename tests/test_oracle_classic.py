"""Pins of the oracle's classic DIC initialisation (all 1-itemsets start in
Dashed Circle, no FirstPass; Algorithm 1, Section 3).

Pinned by a hand-worked trace, by equality of the frequent itemsets with the
FirstPass mode and with exhaustive enumeration, and by the level-wise
structure with one block per pass: the candidates counted at stop t are
C_1 = every item, then textbook apriori-gen of the frequent t-itemsets.
"""
import json
import os

import numpy as np
import pytest

from helpers import apriori_gen, as_dict, items_of, pack

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "classic_hand_example.json")


def _rand_db(seed, n, m, density):
    rng = np.random.default_rng(seed)
    return pack([[i for i in range(m) if rng.random() < density] for _ in range(n)], m)


def test_hand_example(orc):
    g = json.load(open(GOLDEN))
    rows = pack(g["transactions"], g["m"])
    r = orc.dic(rows, g["m"], g["minsup"], g["M"], init_mode=1)
    assert r.trace.tolist() == g["trace"]
    assert [[list(items_of(mk)), int(c)] for mk, c in zip(r.masks, r.counts)] == g["itemsets"]
    assert r.stats["tests"] == g["tests"] and r.stats["stops"] == g["stops"]
    assert r.stats["tau"] == g["tau"] and r.stats["stop_max"] == g["stop_max"]


@pytest.mark.parametrize("seed,n,m,density,minsup,Ms", [
    (1, 200, 10, 0.35, 0.05, (1, 7, 50, 200)),
    (2, 500, 16, 0.25, 0.03, (13, 100, 499)),
    (3, 300, 70, 0.1, 0.02, (30, 300)),
])
def test_same_itemsets_as_firstpass_and_bruteforce(orc, seed, n, m, density, minsup, Ms):
    rows = _rand_db(seed, n, m, density)
    ref = orc.bruteforce(rows, m, minsup) if m <= 20 else orc.tidlist(rows, m, minsup)
    for M in Ms:
        c = orc.dic(rows, m, minsup, M, init_mode=1)
        f = orc.dic(rows, m, minsup, M)
        assert np.array_equal(c.masks, ref.masks) and np.array_equal(c.counts, ref.counts), M
        assert np.array_equal(c.masks, f.masks) and np.array_equal(c.counts, f.counts), M
        # every 1-itemset is created at the start, so classic mode knows all m
        assert c.stats["known"] >= m
        assert c.stats["tests"] >= f.stats["tests"] - n * m


def test_one_block_per_pass_is_levelwise_from_all_items(orc):
    rows = _rand_db(31, 300, 14, 0.45)
    m, ms = 14, 0.06
    r = orc.dic(rows, m, ms, 300, init_mode=1)
    L = as_dict(r.masks, r.counts)
    levels = {}
    for s in L:
        levels.setdefault(len(s), set()).add(s)
    assert r.stats["stop_max"] == 1
    assert int(r.trace[0][2]) == m  # C_1: every item
    for t in range(1, len(r.trace)):
        assert int(r.trace[t][2]) == len(apriori_gen(levels.get(t, set()))), t
    assert len(apriori_gen(levels.get(len(r.trace), set()))) == 0


def test_candgen_modes_agree_in_classic_mode(orc):
    rows = _rand_db(8, 250, 12, 0.4)
    for M in (5, 60):
        a = orc.dic(rows, 12, 0.05, M, candgen_mode=0, init_mode=1)
        b = orc.dic(rows, 12, 0.05, M, candgen_mode=1, init_mode=1)
        assert np.array_equal(a.masks, b.masks) and np.array_equal(a.trace, b.trace)


def test_infrequent_items_are_pruned_or_solid_circles(orc):
    # an item present in 1 of 100 rows can never reach tau = 20: with M = 10
    # its bound 1 + 10 * (10 - stop) falls below 20 at stop 9 at the latest
    rows = pack([[0, 1] if t != 5 else [0, 1, 2] for t in range(100)], 3)
    r = orc.dic(rows, 3, 0.2, 10, init_mode=1)
    assert [list(items_of(mk)) for mk in r.masks] == [[0], [1], [0, 1]]
    assert int(r.trace[:, 4].sum()) >= 1  # item 2 was pruned
