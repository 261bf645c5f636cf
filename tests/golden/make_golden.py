"""Write the expected results of the large workloads, from the CPU oracle alone.

Every expected value here comes from ``oracle.dic`` (and nothing else) run on
the seeded synthetic databases of ``synth``:

    python tests/golden/make_golden.py [2] [3]    single-database workloads
    python tests/golden/make_golden.py batch      all 256 batch databases
    python tests/golden/make_golden.py serve      a seeded served request list

Single-database workloads store a SHA-256 of the input rows (so a test can
confirm it regenerated the same database), the oracle's statistics and
per-stop trace (JSON), and every frequent itemset with its count (gzip text,
one line per itemset: ascending item indices, a tab, the count; canonical
order).

The batch and the served list are too large to store itemset by itemset.  Per
database or request they keep the rows' SHA-256, the oracle's statistics and
``helpers.result_digest`` of its result (canonical masks, counts and per-stop
trace), so a test compares a GPU result with the oracle's bit for bit.

  batch  -- ``synth.batch_specs(256)``: n ~ U{1,000..200,000}, m from
            {64, 256, 1024}, Quest-style, minsup U[1 %, 5 %], M = n // 20.
  serve  -- the resident pool of the serving benchmark (the n = 10^6 x 1,000
            sparse database, the n = 5*10^5 x 128 dense one, 16 batch-shaped
            ones) and the first second of its open-loop Poisson stream at 200
            requests/s (``synth.serve_stream``, default seed), every request
            with its database's own M; plus four fixed minsups on each of the
            two large databases.

The oracle is serial; databases run in parallel worker processes (spawned),
largest first.  The batch takes about 15 minutes on 6 cores, the served list
about 40 (a dense request near minsup 25 % alone takes about 25 minutes).
"""
from __future__ import annotations

import concurrent.futures as cf
import gzip
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402
from helpers import result_digest  # noqa: E402

SERVE_RATE = 200.0
SERVE_SECONDS = 1.0
SERVE_EXTRA = {0: (0.005, 0.01, 0.02, 0.05), 1: (0.25, 0.27, 0.29, 0.30)}
SERVE_RANGES = [(0.005, 0.05), (0.25, 0.30)] + [(0.01, 0.05)] * 16
STAT_KEYS = ("tau", "block", "stop_max", "stops", "tests", "peak_live", "n_frequent", "k_max",
             "known")


def rows_digest(rows: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(rows, dtype="<u8").tobytes()).hexdigest()


def items_of(row) -> list[int]:
    out = []
    for w, x in enumerate(row):
        x = int(x)
        while x:
            b = (x & -x).bit_length() - 1
            out.append(64 * w + b)
            x &= x - 1
    return out


def write(index: int) -> None:
    c = synth.config(index)
    t0 = time.time()
    r = oracle.dic(c["rows"], c["m"], c["minsup"], c["M"])
    dt = time.time() - t0
    base = os.path.join(HERE, f"workload{index}")
    meta = {
        "workload": c["name"], "index": index, "n": int(c["rows"].shape[0]), "m": c["m"],
        "minsup": c["minsup"], "M": c["M"], "rows_sha256": rows_digest(c["rows"]),
        "numpy": np.__version__, "stats": r.stats, "oracle_seconds": round(dt, 1),
        "trace_fields": list(oracle.TRACE_FIELDS), "trace": r.trace.tolist(),
        "source": "oracle.dic on synth.config(%d); written by tests/golden/make_golden.py" % index,
    }
    with open(base + ".json", "w") as f:
        json.dump(meta, f)
    with gzip.open(base + ".itemsets.txt.gz", "wt") as f:
        for row, cnt in zip(r.masks, r.counts):
            f.write(",".join(map(str, items_of(row))) + "\t" + str(int(cnt)) + "\n")
    print(f"workload {index}: |L|={len(r.counts)} stops={r.stats['stops']} "
          f"tests={r.stats['tests']} oracle {dt:.1f}s", flush=True)


# ------------------------------------------------------------------ workers

_ROWS: dict = {}


def _serve_pool_rows(j: int):
    """Rows and M of serving pool database j (0: sparse, 1: dense, 2..: batch
    shaped), generated once per worker."""
    if j not in _ROWS:
        if j == 0:
            c = synth.config(2)
            _ROWS[j] = (c["rows"], c["m"], c["M"])
        elif j == 1:
            c = synth.config(3)
            _ROWS[j] = (c["rows"], c["m"], c["M"])
        else:
            s = synth.batch_specs(16, seed=synth.CONFIG_SEED_BASE + 5)[j - 2]
            _ROWS[j] = (synth.batch_one(s), s["m"], s["M"])
    return _ROWS[j]


def _oracle_entry(rows, m, minsup, M):
    t0 = time.time()
    r = oracle.dic(rows, m, minsup, M)
    dt = time.time() - t0
    return {"rows_sha256": rows_digest(rows), "n": int(rows.shape[0]), "m": int(m),
            "minsup": float(minsup), "M": int(M),
            "stats": {k: int(r.stats[k]) for k in STAT_KEYS},
            "digest": result_digest(r.masks, r.counts, r.trace),
            "oracle_seconds": round(dt, 2)}


def _batch_task(spec):
    rows = synth.batch_one(spec)
    e = _oracle_entry(rows, spec["m"], spec["minsup"], spec["M"])
    e["index"] = spec["index"]
    return e


def _serve_task(req):
    rows, m, M = _serve_pool_rows(req["db"])
    e = _oracle_entry(rows, m, req["minsup"], M)
    e.update({k: req[k] for k in ("id", "db", "t")})
    return e


def _run(tasks, fn, workers):
    out = []
    ctx = mp.get_context("spawn")
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        futs = {ex.submit(fn, t): t for t in tasks}
        for k, f in enumerate(cf.as_completed(futs)):
            e = f.result()
            out.append(e)
            print(f"  [{k + 1}/{len(tasks)}] n={e['n']} m={e['m']} minsup={e['minsup']:.4f} "
                  f"|L|={e['stats']['n_frequent']} oracle {e['oracle_seconds']:.1f}s", flush=True)
    return out


def write_batch(workers: int) -> None:
    specs = synth.batch_specs(256)
    # largest counting work first: the slowest databases do not trail alone
    order = sorted(specs, key=lambda s: -s["n"] * (1 + s["m"] // 64) / s["minsup"])
    t0 = time.time()
    entries = sorted(_run(order, _batch_task, workers), key=lambda e: e["index"])
    doc = {"source": "oracle.dic on every synth.batch_specs(256) database; written by "
                     "tests/golden/make_golden.py batch",
           "recipe": "synth.batch_specs(256), rows from synth.batch_one",
           "digest": "tests/helpers.py result_digest (canonical masks, counts, trace)",
           "numpy": np.__version__, "wall_seconds": round(time.time() - t0, 1),
           "entries": entries}
    with open(os.path.join(HERE, "batch256.json"), "w") as f:
        json.dump(doc, f, indent=0)
    print(f"batch: {len(entries)} databases in {time.time() - t0:.0f}s", flush=True)


def serve_requests():
    """The request list: the stream's first second, then the fixed extras."""
    stream = synth.serve_stream([0] * len(SERVE_RANGES), rate=SERVE_RATE,
                                duration_s=SERVE_SECONDS, minsup_ranges=SERVE_RANGES)
    reqs = [{"id": i, "t": t, "db": j, "minsup": ms} for i, (t, j, ms) in enumerate(stream)]
    for j, mins in SERVE_EXTRA.items():
        for ms in mins:
            reqs.append({"id": len(reqs), "t": None, "db": j, "minsup": ms})
    return reqs


def write_serve(workers: int) -> None:
    reqs = serve_requests()
    pool = []
    for j in range(len(SERVE_RANGES)):
        rows, m, M = _serve_pool_rows(j)
        pool.append({"db": j, "n": int(rows.shape[0]), "m": int(m), "M": int(M),
                     "rows_sha256": rows_digest(rows), "minsup_range": SERVE_RANGES[j]})
    _ROWS.clear()

    def cost(r):  # dense requests near 25 % dominate; then the sparse ones
        return (2 if r["db"] == 1 else 1 if r["db"] == 0 else 0, -r["minsup"])
    t0 = time.time()
    entries = sorted(_run(sorted(reqs, key=cost, reverse=True), _serve_task, workers),
                     key=lambda e: e["id"])
    doc = {"source": "oracle.dic on every request; written by tests/golden/make_golden.py serve",
           "stream": {"rate": SERVE_RATE, "duration_s": SERVE_SECONDS,
                      "seed": synth.CONFIG_SEED_BASE + 5, "recipe": "synth.serve_stream"},
           "extra_minsups": {str(k): v for k, v in SERVE_EXTRA.items()},
           "digest": "tests/helpers.py result_digest (canonical masks, counts, trace)",
           "numpy": np.__version__, "wall_seconds": round(time.time() - t0, 1),
           "pool": pool, "requests": entries}
    with open(os.path.join(HERE, "serve_requests.json"), "w") as f:
        json.dump(doc, f, indent=0)
    print(f"serve: {len(entries)} requests in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    workers = int(os.environ.get("GOLDEN_WORKERS", "6"))
    for a in (sys.argv[1:] or ["3", "2"]):
        if a == "batch":
            write_batch(workers)
        elif a == "serve":
            write_serve(workers)
        else:
            write(int(a))
