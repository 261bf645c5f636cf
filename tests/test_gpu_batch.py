"""Full-size parity for the batch of 256 databases (uneven n and m, W = 1/4/16).

At this size the oracle cannot mine every database in a test, so:
  * every database: the batched result equals mining it alone (itemsets,
    counts, statistics, per-stop trace), is in canonical order, is downward
    closed with non-increasing counts, sampled itemsets recount exactly on the
    CPU, and sampled negative-border itemsets recount below the threshold;
  * the databases with the least counting work: the full oracle result.
"""
import sys

import numpy as np
import pytest

import synth
from helpers import items_of

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same(a, b):
    return (np.array_equal(a.masks, b.masks) and np.array_equal(a.counts, b.counts)
            and np.array_equal(a.trace, b.trace) and a.stats["tests"] == b.stats["tests"])


def _diff(a, b):
    """Which parts of two results differ (for the failure message)."""
    out = []
    if a.masks.shape != b.masks.shape or not np.array_equal(a.masks, b.masks):
        out.append(f"itemsets {a.masks.shape[0]} vs {b.masks.shape[0]}")
    elif not np.array_equal(a.counts, b.counts):
        out.append("counts")
    if a.trace is None or b.trace is None or a.trace.shape != b.trace.shape:
        out.append("trace shape")
    elif not np.array_equal(a.trace, b.trace):
        s = int(np.argwhere((a.trace != b.trace).any(axis=1))[0, 0])
        out.append(f"trace from stop entry {s}: {a.trace[s].tolist()} vs {b.trace[s].tolist()}")
    if a.stats["tests"] != b.stats["tests"]:
        out.append("tests")
    return "; ".join(out)


def test_batch_of_256_full_size(orc):
    import paper_1812_10959_amd as dic
    _say("generating 256 databases")
    spec = synth.batch_config(256)
    dbs = [dic.dic_load_db(d["rows"], d["m"]) for d in spec]
    ms = [d["minsup"] for d in spec]
    Ms = [d["M"] for d in spec]
    _say("batched")
    batched = dic.dic_batch(dbs, ms, Ms)
    rng = np.random.default_rng(4)
    for i, (d, r) in enumerate(zip(spec, batched)):
        solo = dic.dic_mine(dbs[i], ms[i], Ms[i])
        assert _same(r, solo), (i, _diff(r, solo))
        n, m = d["rows"].shape[0], d["m"]
        tau = orc.tau(ms[i], n)
        assert r.stats["tau"] == tau
        L = {items_of(row): int(c) for row, c in zip(r.masks, r.counts)}
        keys = list(L)
        # canonical order
        ks = [(len(t), t) for t in keys]
        assert ks == sorted(ks), i
        # downward closure, counts non-increasing
        for t, c in L.items():
            if len(t) > 1:
                for x in range(len(t)):
                    sub = t[:x] + t[x + 1:]
                    assert sub in L and L[sub] >= c, (i, t)
        # exact recount of sampled itemsets
        pick = rng.choice(len(keys), size=min(6, len(keys)), replace=False)
        masks = r.masks[pick]
        got = orc.count_block(d["rows"], m, masks)
        assert got.tolist() == [L[keys[j]] for j in pick], i
        # negative border sample: extensions of frequent itemsets by a frequent
        # item whose maximal subsets are all frequent but which are not in L
        singles = sorted(t[0] for t in keys if len(t) == 1)
        border = []
        for j in rng.permutation(len(keys))[:40]:
            t = keys[j]
            for it in rng.permutation(singles)[:6]:
                it = int(it)
                if it in t:
                    continue
                c = tuple(sorted(t + (it,)))
                if c not in L and all(c[:x] + c[x + 1:] in L for x in range(len(c))):
                    border.append(c)
        if border:
            W = d["rows"].shape[1]
            bm = np.zeros((len(border), W), np.uint64)
            for b, c in enumerate(border):
                for p in c:
                    bm[b, p >> 6] |= np.uint64(1) << np.uint64(p & 63)
            assert (orc.count_block(d["rows"], m, bm) < tau).all(), i
    # full oracle on the databases with the least counting work
    order = np.argsort([r.stats["tests"] for r in batched])[:10]
    for i in order:
        d = spec[i]
        _say(f"oracle db {i}: n={d['rows'].shape[0]} m={d['m']} tests={batched[i].stats['tests']}")
        ref = orc.dic(d["rows"], d["m"], ms[i], Ms[i])
        assert np.array_equal(batched[i].masks, ref.masks)
        assert np.array_equal(batched[i].counts, ref.counts)
        if ref.trace is None:  # fewer than two frequent items: no stop at all
            assert batched[i].trace is None and batched[i].stats["stops"] == 0
        else:
            assert np.array_equal(batched[i].trace.astype(np.uint64), ref.trace)
