"""Full-size parity for the batch of 256 databases (uneven n and m, W = 1/4/16).

Every database's result -- mined in one batch, and mined alone -- equals the
CPU oracle's bit for bit: the same itemsets in canonical order, the same
counts, the same per-stop trace and statistics.  The oracle's results were
written by ``tests/golden/make_golden.py batch`` (oracle only, about 100 CPU
minutes) as SHA-256 digests (``helpers.result_digest``) with the statistics
and the SHA-256 of each regenerated database.  The batch also runs with HIP
graphs off and with a second launch grid: the results must not move.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import synth
from helpers import result_digest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch256.json")
STAT_KEYS = ("tau", "block", "stop_max", "stops", "tests", "peak_live", "n_frequent", "k_max",
             "known")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check_all(results, golden, label):
    bad = []
    for i, (r, g) in enumerate(zip(results, golden)):
        got = result_digest(r.masks, r.counts, r.trace)
        stats = {k: int(r.stats[k]) for k in STAT_KEYS}
        if got != g["digest"] or stats != g["stats"]:
            bad.append((i, {k: (stats[k], g["stats"][k]) for k in STAT_KEYS
                            if stats[k] != g["stats"][k]}))
    assert not bad, f"{label}: {len(bad)} databases differ from the oracle, first {bad[:3]}"


@pytest.fixture(scope="module")
def batch():
    import paper_1812_10959_amd as dic
    golden = json.load(open(GOLDEN))["entries"]
    assert len(golden) == 256
    # generated serially in this process (about two minutes): a worker pool
    # would be started from a process that may hold a GPU context
    spec, dbs = [], []
    for i, (s, g) in enumerate(zip(synth.batch_specs(256), golden)):
        rows = synth.batch_one(s)
        h = hashlib.sha256(np.ascontiguousarray(rows, dtype="<u8").tobytes()).hexdigest()
        assert h == g["rows_sha256"] and s["M"] == g["M"], f"database {i} was not regenerated"
        spec.append({"m": s["m"], "minsup": s["minsup"], "M": s["M"]})
        dbs.append(dic.dic_load_db(rows, s["m"]))
        if i % 32 == 31:
            _say(f"  {i + 1} of 256 databases generated and loaded")
    return dic, spec, dbs, golden


def test_batch_of_256_equals_oracle(batch):
    dic, spec, dbs, golden = batch
    _say("batched")
    res = dic.dic_batch(dbs, [d["minsup"] for d in spec], [d["M"] for d in spec])
    _check_all(res, golden, "batched")


def test_solo_runs_equal_oracle(batch):
    dic, spec, dbs, golden = batch
    _say("solo")
    res = [dic.dic_mine(db, d["minsup"], d["M"]) for db, d in zip(dbs, spec)]
    _check_all(res, golden, "solo")


@pytest.mark.parametrize("graphs,grid", [(0, 2048), (1, 1024)])
def test_batch_graphs_and_grid_do_not_change_results(batch, graphs, grid):
    dic, spec, dbs, golden = batch
    _say(f"batched, graphs {graphs}, grid {grid}")
    try:
        dic.dic_set_option("graphs", graphs)
        dic.dic_set_option("count_grid", grid)
        res = dic.dic_batch(dbs, [d["minsup"] for d in spec], [d["M"] for d in spec])
    finally:
        dic.dic_set_option("graphs", 1)
        dic._apply_tuning()
    _check_all(res, golden, f"graphs {graphs} grid {grid}")
