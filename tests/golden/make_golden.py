"""Write the expected results of the large single-database workloads.

Runs the CPU oracle (and nothing else) on the seeded synthetic databases and
stores, per workload: a SHA-256 of the input rows (so a test can confirm it
regenerated the same database), the oracle's statistics and per-stop trace
(JSON), and every frequent itemset with its count (gzip text, one line per
itemset: ascending item indices, a tab, the count; canonical order).

    python tests/golden/make_golden.py [index ...]      (default: 2 3)

The oracle takes minutes on these sizes; the files are committed.
"""
from __future__ import annotations

import gzip
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


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


if __name__ == "__main__":
    for a in (sys.argv[1:] or ["3", "2"]):
        write(int(a))
