"""Served requests equal the oracle, request by request, under overlap.

The request list is the serving benchmark's workload: one second of Poisson
arrivals at 200 requests/s over the resident pool (the n = 10^6 x 1,000 sparse
database, the n = 5 x 10^5 x 128 dense one and 16 batch-shaped databases),
each request with its own minsup, followed by fixed extras at the ends of the
two big databases' minsup ranges.  ``tests/golden/make_golden.py serve`` mined
every request with the CPU oracle alone and stored a SHA-256 digest of the
canonical result (``helpers.result_digest``) with the statistics.  Here the
same list is replayed into one server at the stream's own arrival times, so
requests join and leave the running batch while others are mid-flight; every
result, and every request's stop trace, must equal the oracle's.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np
import pytest

import synth
from helpers import result_digest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "serve_requests.json")
STAT_KEYS = ("tau", "block", "stop_max", "stops", "tests", "peak_live", "n_frequent", "k_max",
             "known")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pool_rows(j: int):
    """The pool's database j, as the golden's writer made it (0: the sparse
    headline database, 1: the dense one, 2..17: batch-shaped)."""
    if j == 0:
        c = synth.config(2)
        return c["rows"], c["m"], c["M"]
    if j == 1:
        c = synth.config(3)
        return c["rows"], c["m"], c["M"]
    s = synth.batch_specs(16, seed=synth.CONFIG_SEED_BASE + 5)[j - 2]
    return synth.batch_one(s), s["m"], s["M"]


@pytest.fixture(scope="module")
def served():
    import paper_1812_10959_amd as dic
    doc = json.load(open(GOLDEN))
    dbs = []
    for p in doc["pool"]:
        rows, m, M = _pool_rows(p["db"])
        h = hashlib.sha256(np.ascontiguousarray(rows, dtype="<u8").tobytes()).hexdigest()
        assert h == p["rows_sha256"] and M == p["M"], f"pool database {p['db']} differs"
        dbs.append(dic.dic_load_db(rows, m))
    _say(f"pool of {len(dbs)} loaded")
    return dic, doc, dbs


def _replay(dic, doc, dbs, max_active):
    reqs = doc["requests"]
    srv = dic.dic_serve_create(200 << 30, max_active=max_active)
    tickets = []
    t0 = time.perf_counter()
    for r in reqs:
        if r["t"] is not None:
            wait = r["t"] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
        tickets.append(dic.dic_serve_submit(srv, dbs[r["db"]], r["minsup"], r["M"]))
    _say(f"submitted {len(tickets)} in {time.perf_counter() - t0:.2f}s")
    out = [dic.dic_serve_wait(srv, t, 120_000) for t in tickets]
    _say(f"served in {time.perf_counter() - t0:.2f}s")
    dic.dic_serve_destroy(srv)
    return out


def _check(out, doc):
    bad = []
    for r, g in zip(out, doc["requests"]):
        stats = {k: int(r.stats[k]) for k in STAT_KEYS}
        if result_digest(r.masks, r.counts, r.trace) != g["digest"] or stats != g["stats"]:
            bad.append((g["id"], g["db"], g["minsup"],
                        {k: (stats[k], g["stats"][k]) for k in STAT_KEYS
                         if stats[k] != g["stats"][k]}))
    assert not bad, f"{len(bad)} of {len(out)} served requests differ, first {bad[:3]}"


@pytest.mark.parametrize("max_active", [64, 4])
def test_served_stream_equals_oracle(served, max_active):
    dic, doc, dbs = served
    _say(f"replay, max_active {max_active}")
    _check(_replay(dic, doc, dbs, max_active), doc)
