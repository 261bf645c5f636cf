"""Test-side helpers: item lists <-> packed rows, result comparison, pure-Python checks.

Nothing here is imported by the GPU library or by the oracle.
"""
from __future__ import annotations

import itertools

import numpy as np


def pack(item_lists, m):
    """Item lists -> uint64[n, W] rows (item p at bit p&63 of word p>>6)."""
    W = (m + 63) // 64
    rows = np.zeros((len(item_lists), W), np.uint64)
    for r, items in enumerate(item_lists):
        for p in items:
            rows[r, p >> 6] |= np.uint64(1) << np.uint64(p & 63)
    return rows


def items_of(mask_row):
    out = []
    for w, x in enumerate(mask_row):
        x = int(x)
        while x:
            b = (x & -x).bit_length() - 1
            out.append(64 * w + b)
            x &= x - 1
    return tuple(out)


def as_dict(masks, counts):
    """{item tuple: count}."""
    return {items_of(masks[i]): int(counts[i]) for i in range(len(counts))}


def canonical_key(items):
    return (len(items), tuple(items))


def is_canonical(masks):
    keys = [canonical_key(items_of(r)) for r in masks]
    return all(keys[i] < keys[i + 1] for i in range(len(keys) - 1))


def py_support(rows_sets, itemset):
    s = set(itemset)
    return sum(1 for t in rows_sets if s <= t)


def py_bruteforce(item_lists, m, tau):
    """Pure-Python enumeration of every itemset; tiny inputs only."""
    rows_sets = [set(t) for t in item_lists]
    out = {}
    for k in range(1, m + 1):
        any_k = False
        for c in itertools.combinations(range(m), k):
            s = py_support(rows_sets, c)
            if s >= tau:
                out[c] = s
                any_k = True
        if not any_k:
            break  # anti-monotone: no frequent k-set, no frequent (k+1)-set
    return out


def apriori_gen(level_sets):
    """Textbook candidate generation from frequent k-itemsets (sorted tuples):
    join pairs sharing the first k-1 items, keep those whose k-subsets are all
    frequent."""
    L = sorted(level_sets)
    S = set(L)
    out = set()
    for i in range(len(L)):
        for j in range(i + 1, len(L)):
            a, b = L[i], L[j]
            if a[:-1] != b[:-1]:
                continue
            c = a + (b[-1],) if a[-1] < b[-1] else b + (a[-1],)
            if all(c[:x] + c[x + 1:] in S for x in range(len(c))):
                out.add(c)
    return out


def unpack_bool(rows, m):
    n, W = rows.shape
    return np.unpackbits(rows.astype("<u8").view(np.uint8).reshape(n, W * 8), axis=1,
                         bitorder="little")[:, :m].astype(bool)


def np_support(rows, m, itemsets):
    """numpy recount of each itemset (tuple of items) over all rows."""
    b = unpack_bool(rows, m)
    return np.array([int(np.all(b[:, list(s)], axis=1).sum()) for s in itemsets], np.int64)


def result_digest(masks, counts, trace) -> str:
    """SHA-256 of a mining result in canonical order: the masks (uint64 LE,
    |L| x W), the counts (uint32 LE) and the per-stop trace's seven fields
    (uint64 LE, stops x 7; empty when no stop ran).  Equal digests mean the
    same itemsets, counts and trace bit for bit."""
    import hashlib
    h = hashlib.sha256()
    h.update(b"masks")
    h.update(np.ascontiguousarray(masks, dtype="<u8").tobytes())
    h.update(b"counts")
    h.update(np.ascontiguousarray(counts, dtype="<u4").tobytes())
    h.update(b"trace")
    if trace is not None and len(trace):
        h.update(np.ascontiguousarray(np.asarray(trace)[:, :7], dtype="<u8").tobytes())
    return h.hexdigest()
