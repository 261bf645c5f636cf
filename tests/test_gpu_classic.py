"""GPU classic DIC initialisation (option "init" = 1) and Apriori mode
(M >= n) against the oracle.

Classic mode starts with every 1-itemset as a dashed circle (Algorithm 1)
instead of FirstPass; itemsets, counts, statistics and the per-stop trace
must equal the oracle's classic mode bit for bit, in both counting layouts.
With M >= n each stop is a full pass: the run is level-wise Apriori, and the
per-stop live counts are apriori-gen's candidate counts (the oracle's
trace, pinned to an independent apriori-gen).
"""
import json
import os
import sys

import numpy as np
import pytest

import synth
from helpers import apriori_gen, as_dict, items_of, pack

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
STAT_KEYS = ("tau", "block", "stop_max", "stops", "tests", "peak_live", "n_frequent", "k_max",
             "known")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same(g, r, label):
    assert g.masks.shape == r.masks.shape, (label, g.masks.shape, r.masks.shape)
    assert np.array_equal(g.masks, r.masks), label
    assert np.array_equal(g.counts, r.counts), label
    for k in STAT_KEYS:
        assert g.stats[k] == r.stats[k], (label, k, g.stats[k], r.stats[k])
    if r.trace is None:
        assert g.trace is None or len(g.trace) == 0, label
    else:
        assert np.array_equal(g.trace.astype(np.uint64), r.trace), label


def _mine(dic, db, minsup, M, init, layout=1):
    dic.dic_set_option("init", init)
    dic.dic_set_option("layout", layout)
    try:
        return dic.dic_mine(db, minsup, M)
    finally:
        dic.dic_set_option("init", 0)
        dic.dic_set_option("layout", 1)


def test_hand_example(orc):
    import paper_1812_10959_amd as dic
    g = json.load(open(os.path.join(GOLDEN, "classic_hand_example.json")))
    rows = pack(g["transactions"], g["m"])
    db = dic.dic_load_db(rows, g["m"])
    for layout in (1, 0):
        r = _mine(dic, db, g["minsup"], g["M"], 1, layout)
        assert r.trace.tolist() == g["trace"], layout
        assert [[list(items_of(mk)), int(c)] for mk, c in zip(r.masks, r.counts)] == g["itemsets"]
        assert r.stats["tests"] == g["tests"] and r.stats["stops"] == g["stops"]


@pytest.mark.parametrize("seed,n,m,density,minsup,Ms", [
    (1, 400, 12, 0.35, 0.05, (1, 9, 60, 400)),
    (2, 3000, 70, 0.12, 0.03, (150, 1000, 3000)),
    (3, 2000, 200, 0.06, 0.02, (100, 700)),
    (4, 1500, 1000, 0.01, 0.01, (300, 1500)),
])
def test_random_databases(orc, seed, n, m, density, minsup, Ms):
    import paper_1812_10959_amd as dic
    rows = synth.uniform_random(n, m, density, seed=4400 + seed)
    db = dic.dic_load_db(rows, m)
    for M in Ms:
        ref = orc.dic(rows, m, minsup, M, init_mode=1)
        first = orc.dic(rows, m, minsup, M)
        assert np.array_equal(ref.masks, first.masks)
        for layout in (1, 0):
            _say(f"classic seed={seed} n={n} m={m} M={M} layout={layout} |L|={len(ref.counts)}")
            _same(_mine(dic, db, minsup, M, 1, layout), ref, (seed, M, layout))


def test_config1_classic(orc):
    import paper_1812_10959_amd as dic
    c = synth.config(1)
    db = dic.dic_load_db(c["rows"], c["m"])
    ref = orc.dic(c["rows"], c["m"], c["minsup"], c["M"], init_mode=1)
    _say(f"config 1 classic: stops={ref.stats['stops']} tests={ref.stats['tests']}")
    _same(_mine(dic, db, c["minsup"], c["M"], 1), ref, "config1 classic")


@pytest.mark.parametrize("init", [0, 1])
def test_apriori_mode(orc, init):
    """M >= n: one block per pass, so each stop counts one Apriori level."""
    import paper_1812_10959_amd as dic
    n, m = 2000, 24
    rows = synth.uniform_random(n, m, 0.3, seed=4500 + init)
    db = dic.dic_load_db(rows, m)
    g = _mine(dic, db, 0.04, 10 * n, init)
    _same(g, orc.dic(rows, m, 0.04, 10 * n, init_mode=init), f"apriori init={init}")
    assert g.stats["stop_max"] == 1
    levels = {}
    for s in as_dict(g.masks, g.counts):
        levels.setdefault(len(s), set()).add(s)
    live = [int(x) for x in g.trace[:, 2]]
    # counted candidates per level: C_1 = every item (classic) and C_k = apriori-gen(L_{k-1})
    want = ([m] if init else []) + [len(apriori_gen(levels.get(k, set())))
                                    for k in range(1, len(live) + (0 if init else 1))]
    assert live == want[:len(live)] and len(live) == len(want), (live, want)


def test_batch_classic_equals_solo(orc):
    import paper_1812_10959_amd as dic
    spec = synth.batch_config(12, seed=4600)
    dbs = [dic.dic_load_db(d["rows"], d["m"]) for d in spec]
    ms = [d["minsup"] for d in spec]
    Ms = [d["M"] for d in spec]
    dic.dic_set_option("init", 1)
    try:
        batched = dic.dic_batch(dbs, ms, Ms)
        solo = [dic.dic_mine(dbs[i], ms[i], Ms[i]) for i in range(len(spec))]
    finally:
        dic.dic_set_option("init", 0)
    order = np.argsort([r.stats["tests"] for r in batched])
    for i in range(len(spec)):
        assert np.array_equal(batched[i].masks, solo[i].masks), i
        assert np.array_equal(batched[i].counts, solo[i].counts), i
        assert np.array_equal(batched[i].trace, solo[i].trace), i
    for i in order[:3]:
        d = spec[i]
        _say(f"oracle classic db {i}: n={d['rows'].shape[0]} m={d['m']}")
        _same(batched[i], orc.dic(d["rows"], d["m"], ms[i], Ms[i], init_mode=1), f"db {i}")
