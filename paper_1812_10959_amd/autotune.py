"""Autotuner for the count kernels' planning knobs.

The knobs (``dic_set_option``) decide how a stop's counting work is cut into
workgroups and tiles:

* ``vt_target``      workgroups aimed at per job per stop (item bitsets);
  more candidates per thread are used once the work exceeds it;
* ``vt_wave_k``      live-candidate count below which one wave counts each
  candidate over the whole block, with no LDS tile;
* ``vt_tile_words``  64-row words per LDS tile (tile shape: frequent items
  x words);
* ``count_grid``     workgroups launched for the count kernels (blocks in
  flight per CU).

No setting changes any result.  ``tune`` times each workload of a sample
under each combination (after a warm-up), checks that every combination
returns exactly the same itemsets, counts and traces, and picks the
combination with the lowest mean of per-workload time ratios to the
defaults (so a long workload does not outweigh a short one).  ``save``
writes the choice to JSON; the package applies ``tuning.json`` beside it at
import.

    python -m paper_1812_10959_amd.autotune --batch 48 --out paper_1812_10959_amd/tuning.json
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_JSON = os.path.join(HERE, "tuning.json")

DEFAULTS = {"vt_target": 768, "vt_wave_k": 2048, "vt_tile_words": 16, "count_grid": 2048}
GRID = {
    "vt_target": (384, 512, 640, 768, 1024),
    "vt_wave_k": (2048, 8192, 16384),
    "vt_tile_words": (8, 16),
    "count_grid": (1024, 2048),
}


def apply(settings: dict) -> None:
    from . import dic_set_option
    for k, v in settings.items():
        dic_set_option(k, int(v))


def _run_one(dic, item):
    kind, payload = item
    if kind == "mine":
        db, ms, M = payload
        return [dic.dic_mine(db, ms, M)]
    dbs, ms, Ms = payload
    return list(dic.dic_batch(dbs, ms, Ms))


def _run(dic, work):
    """Mine every (kind, payload) item; returns results in order."""
    out = []
    for item in work:
        out.extend(_run_one(dic, item))
    return out


def _timed(dic, work, reps):
    """Per-item median seconds over reps, and the results of the last rep."""
    times, res = [], []
    for item in work:
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            r = _run_one(dic, item)
            ts.append(time.perf_counter() - t0)
        times.append(float(np.median(ts)))
        res.extend(r)
    return times, res


def _same(a, b):
    return all(np.array_equal(x.masks, y.masks) and np.array_equal(x.counts, y.counts)
               and ((x.trace is None and y.trace is None) or np.array_equal(x.trace, y.trace))
               for x, y in zip(a, b))


def tune(work, grid=GRID, reps: int = 2, log=print) -> dict:
    """work: list of ("mine", (db, minsup, M)) and ("batch", (dbs, minsups, Ms)).

    Returns {"best": settings, "seconds": best time, "default_seconds": ...,
    "table": [(settings, seconds), ...]}."""
    import paper_1812_10959_amd as dic
    apply(DEFAULTS)
    _run(dic, work)  # warm graphs and caches
    base, ref = _timed(dic, work, reps)
    names = list(grid)
    table = []
    for combo in itertools.product(*(grid[n] for n in names)):
        settings = dict(zip(names, combo))
        apply(settings)
        _run(dic, work)  # warm-up under these settings
        times, res = _timed(dic, work, reps)
        if not _same(res, ref):
            apply(DEFAULTS)
            raise AssertionError(f"settings {settings} changed a result")
        score = float(np.mean([t / b for t, b in zip(times, base)]))
        table.append((settings, score, times))
        log(f"  {settings}: score {score:.4f}, " +
            ", ".join(f"{t * 1e3:.2f} ms" for t in times))
    best, best_score, best_times = min(table, key=lambda kv: kv[1])
    apply(best)
    return {"best": best, "score": best_score, "seconds": best_times, "default_seconds": base,
            "table": [[s, sc, t] for s, sc, t in table]}


def save(result: dict, path: str = TUNING_JSON, workload: str = "") -> None:
    doc = {"settings": result["best"], "score": result["score"], "seconds": result["seconds"],
           "default_seconds": result["default_seconds"], "workload": workload,
           "table": result["table"]}
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)


def load(path: str = TUNING_JSON) -> dict | None:
    """Apply a saved choice; returns it (None when there is no file)."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        doc = json.load(f)
    apply(doc["settings"])
    return doc["settings"]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--batch", type=int, default=48, help="databases of the batch sample")
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--out", default=TUNING_JSON)
    a = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    import synth
    c2 = synth.config(2)
    spec = synth.batch_config(a.batch, workers=16)
    import paper_1812_10959_amd as dic
    db2 = dic.dic_load_db(c2["rows"], c2["m"])
    dbs = [dic.dic_load_db(d["rows"], d["m"]) for d in spec]
    work = [("mine", (db2, c2["minsup"], c2["M"])),
            ("batch", (dbs, [d["minsup"] for d in spec], [d["M"] for d in spec]))]
    res = tune(work, reps=a.reps, log=lambda *x: print(*x, flush=True))
    save(res, a.out, workload=f"n=1e6 m=1000 mine + batch of {a.batch}")
    print(json.dumps({"best": res["best"], "score": res["score"],
                      "ms": [t * 1e3 for t in res["seconds"]],
                      "default_ms": [t * 1e3 for t in res["default_seconds"]]}))


if __name__ == "__main__":
    main()
