"""Full-size parity on the large single-database workloads.

Expected results were written by tests/golden/make_golden.py, which runs only
the CPU oracle (minutes per workload).  The GPU runs in the configuration the
benchmark times (dic_mine, default layout) and also with row bitmaps; every
itemset, count, statistic and per-stop trace entry must match.
"""
import gzip
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(index):
    meta = json.load(open(os.path.join(GOLDEN, f"workload{index}.json")))
    items, counts = [], []
    with gzip.open(os.path.join(GOLDEN, f"workload{index}.itemsets.txt.gz"), "rt") as f:
        for ln in f:
            a, c = ln.rstrip("\n").split("\t")
            items.append([int(x) for x in a.split(",")])
            counts.append(int(c))
    return meta, items, np.array(counts, np.uint32)


def _masks(items, W):
    out = np.zeros((len(items), W), np.uint64)
    for r, it in enumerate(items):
        for p in it:
            out[r, p >> 6] |= np.uint64(1) << np.uint64(p & 63)
    return out


@pytest.mark.parametrize("index", [3, 2])
def test_workload_matches_golden(index):
    import paper_1812_10959_amd as dic
    meta, items, counts = _load(index)
    c = synth.config(index)
    digest = hashlib.sha256(np.ascontiguousarray(c["rows"], dtype="<u8").tobytes()).hexdigest()
    assert digest == meta["rows_sha256"], "regenerated input differs from the golden input"
    W = c["rows"].shape[1]
    want = _masks(items, W)
    db = dic.dic_load_db(c["rows"], c["m"])
    for layout in (1, 0):
        print(f"workload {index} layout {layout}", flush=True)
        dic.dic_set_option("layout", layout)
        try:
            g = dic.dic_mine(db, c["minsup"], c["M"])
        finally:
            dic.dic_set_option("layout", 1)
        assert np.array_equal(g.masks, want)
        assert np.array_equal(g.counts, counts)
        for k in ("tau", "stop_max", "stops", "tests", "peak_live", "n_frequent", "k_max", "known"):
            assert g.stats[k] == meta["stats"][k], k
        assert g.trace.tolist() == meta["trace"]
