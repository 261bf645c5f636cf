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
  flight per CU);
* ``cell:<b>:<k>``   per-shape cells: for stops whose block has words in
  band b and whose survivors are in band k (``tune_cell`` in the library),
  one wave per candidate (mode 1) or LDS tiles with a given workgroup target
  (mode 2), overriding the two global choices above.

No setting changes any result.  Two stages:

1. ``tune`` times each workload of a sample under each combination of the
   global knobs (after a warm-up), checks that every combination returns
   exactly the same itemsets, counts and traces, and keeps the combination
   with the lowest mean of per-workload time ratios to the defaults.
2. ``tune_cells`` mines single databases of several shapes with profiling
   on, once with every stop forced to wave mode and once per tile target.
   Every stop's launch is timed with HIP events; a stop's plan depends only
   on its own cell, and the stops (and their survivor counts) are the same
   under every setting, so each cell takes the setting with the least total
   time over the stops that fall in it.  The cells are kept only if the
   sample (the mines and the batch) is not slower with them, by the same
   measure as stage 1: the mean of the per-workload time ratios.

``save`` writes the choice to JSON; the package applies ``tuning.json``
beside it at import.

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
    "vt_wave_k": (512, 1024, 2048, 4096),
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


TUNE_BB, TUNE_KB = 5, 5
CELL_TARGETS = (256, 384, 512, 768, 1024, 1536)


def tune_cell(block_words: int, K: int) -> tuple:
    """The library's cell of a stop (same bands as tune_cell in C)."""
    b = next((i for i, lim in enumerate((4, 16, 64, 256)) if block_words <= lim), 4)
    k = next((i for i, lim in enumerate((256, 1024, 4096, 16384)) if K < lim), 4)
    return b, k


def apply_cells(cells: dict) -> None:
    """cells: {"b:k": [mode, target]}; clears every other cell."""
    from . import dic_set_option
    dic_set_option("cells_clear", 1)
    for key, (mode, target) in cells.items():
        dic_set_option(f"cell:{key}", int(mode) * 65536 + int(target))


def _stop_cells(r) -> list:
    """(cell, launch ns) of every stop of a profiled result.  The survivors
    planned at stop e are the stop's live candidates minus the ones made in
    the same launch for stop e-1's new boxes."""
    out = []
    if r.trace is None:  # no frequent pair of items: the run had no stop
        return out
    Mp = r.stats["block"]
    for e in range(r.trace.shape[0]):
        stop, rows, live = (int(x) for x in r.trace[e, :3])
        gen_prev = int(r.trace[e - 1, 5]) if e else 0
        K = live - gen_prev
        first = (stop - 1) * Mp
        last = first + rows
        words = ((last - 1) >> 6) - (first >> 6) + 1
        out.append((tune_cell(words, K), int(r.launch_ns[e])))
    return out


def tune_cells(mines, reps: int = 2, log=print, bands=None) -> dict:
    """mines: list of (db, minsup, M); bands: the block bands given cells (all
    when None).  Returns {"cells": {...}, "table": ...}."""
    import paper_1812_10959_amd as dic
    settings = [("wave", {"vt_wave_k": 1 << 30}, [1, 0])]
    settings += [(f"tile{t}", {"vt_wave_k": 0, "vt_target": t}, [2, t]) for t in CELL_TARGETS]
    saved = {k: v for k, v in DEFAULTS.items()}
    apply_cells({})
    totals = {}  # cell -> setting name -> [ns, stops]
    ref = None
    try:
        for name, knobs, _ in settings:
            apply(knobs)
            dic.dic_set_option("profile", 1)
            res = []
            for db, ms, M in mines:
                runs = [dic.dic_mine(db, ms, M) for _ in range(reps)]
                res.append(runs[0])
                per = [_stop_cells(x) for x in runs]
                for e in range(len(per[0])):
                    cell = per[0][e][0]
                    ns = float(np.median([p[e][1] for p in per]))
                    t = totals.setdefault(cell, {}).setdefault(name, [0.0, 0])
                    t[0] += ns
                    t[1] += 1
            dic.dic_set_option("profile", 0)
            if ref is None:
                ref = res
            elif not _same(res, ref):
                raise AssertionError(f"setting {name} changed a result")
            log(f"  {name}: " + ", ".join(
                f"{int(x.launch_ns.astype(np.int64).sum()) / 1e6:.2f} ms"
                for x in res if x.launch_ns is not None))
    finally:
        dic.dic_set_option("profile", 0)
        apply(saved)
    modes = {name: mt for name, _, mt in settings}
    cells, table = {}, {}
    for (b, k), per in sorted(totals.items()):
        if bands is not None and b not in bands:
            continue
        best = min(per, key=lambda nm: per[nm][0])
        cells[f"{b}:{k}"] = modes[best]
        table[f"{b}:{k}"] = {nm: [round(v[0] / 1e6, 4), v[1]] for nm, v in per.items()}
        log(f"  cell {b}:{k}: {best} ({per[best][1]} stops, "
            f"{per[best][0] / 1e6:.3f} ms vs wave {per['wave'][0] / 1e6:.3f} ms)")
    return {"cells": cells, "table": table}


def save(result: dict, path: str = TUNING_JSON, workload: str = "", cells: dict | None = None,
         cell_table: dict | None = None, verify: dict | None = None) -> None:
    doc = {"settings": result["best"], "cells": cells or {}, "score": result["score"],
           "seconds": result["seconds"], "default_seconds": result["default_seconds"],
           "workload": workload, "verify": verify or {}, "cell_table": cell_table or {},
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
    apply_cells(doc.get("cells", {}))
    return doc["settings"]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--batch", type=int, default=48, help="databases of the batch sample")
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--out", default=TUNING_JSON)
    ap.add_argument("--cells-only", action="store_true",
                    help="keep the saved global knobs; retune the per-shape cells")
    ap.add_argument("--cell-bands", default="",
                    help="block bands given cells, e.g. 0,1,2 (default: all)")
    a = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    import synth
    c1, c2, c3 = synth.config(1), synth.config(2), synth.config(3)
    spec = synth.batch_config(a.batch, workers=16)
    solo = synth.batch_config(24, seed=synth.CONFIG_SEED_BASE + 7, workers=16)
    import paper_1812_10959_amd as dic
    log = lambda *x: print(*x, flush=True)  # noqa: E731
    db1, db2, db3 = (dic.dic_load_db(c["rows"], c["m"]) for c in (c1, c2, c3))
    dbs = [dic.dic_load_db(d["rows"], d["m"]) for d in spec]
    sdbs = [dic.dic_load_db(d["rows"], d["m"]) for d in solo]
    work = [("mine", (db2, c2["minsup"], c2["M"])), ("mine", (db3, c3["minsup"], c3["M"])),
            ("batch", (dbs, [d["minsup"] for d in spec], [d["M"] for d in spec]))]
    if a.cells_only and os.path.exists(a.out):
        with open(a.out) as f:
            old = json.load(f)
        res = {k: old[k] for k in ("score", "seconds", "default_seconds", "table")}
        res["best"] = old["settings"]
    else:
        apply_cells({})
        res = tune(work, reps=a.reps, log=log)
        save(res, a.out, workload="global knobs only (per-shape cells pending)")
    apply(res["best"])
    log("per-shape cells ...")
    mines = [(db1, c1["minsup"], c1["M"]), (db2, c2["minsup"], c2["M"]),
             (db3, c3["minsup"], c3["M"])] + [(d, s["minsup"], s["M"]) for d, s in zip(sdbs, solo)]
    bands = {int(x) for x in a.cell_bands.split(",")} if a.cell_bands else None
    cres = tune_cells(mines, reps=a.reps, log=log, bands=bands)
    # keep the cells only if the sample is not slower with them
    apply_cells({})
    _run(dic, work)
    t_without, ref = _timed(dic, work, 9)
    apply_cells(cres["cells"])
    _run(dic, work)
    t_with, res_with = _timed(dic, work, 9)
    assert _same(res_with, ref), "per-shape cells changed a result"
    keep = sum(w / o for w, o in zip(t_with, t_without)) <= len(t_with)
    verify = {"seconds_without_cells": t_without, "seconds_with_cells": t_with, "kept": keep,
              "work": ["mine n=1e6 m=1000", "mine n=5e5 m=128", f"batch of {a.batch}"]}
    log(f"with cells {[round(t * 1e3, 2) for t in t_with]} ms, without "
        f"{[round(t * 1e3, 2) for t in t_without]} ms: {'kept' if keep else 'dropped'}")
    save(res, a.out, workload=f"n=1e6 m=1000 and n=5e5 m=128 mines + batch of {a.batch}",
         cells=cres["cells"] if keep else {}, cell_table=cres["table"], verify=verify)
    print(json.dumps({"best": res["best"], "cells": cres["cells"] if keep else {},
                      "verify": verify}))


if __name__ == "__main__":
    main()
