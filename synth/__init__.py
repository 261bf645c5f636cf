"""Seeded synthetic transaction databases.

Input generation only: every function here draws random databases (or random
request streams) and returns them in the layout the miners consume, a row-major
``uint64[n, W]`` array with ``W = ceil(m / 64)``, item ``p`` stored at bit
``p & 63`` of word ``p >> 6`` and every bit at or above ``m`` zero (the direct
bit representation of Section 4.1, widened from one word to W words).

Nothing in this module counts supports, applies thresholds or builds itemsets:
it is shared by the CPU oracle and the GPU path for exactly that reason, so
that both read the same inputs while sharing no step of the method.

The generators are written from parameter lists, not from any existing
generator's source:

* ``quest`` -- a Quest-style basket generator: latent patterns with Poisson
  lengths, exponential weights and a per-pattern corruption level; each
  transaction draws weighted patterns and keeps each pattern item with
  probability ``1 - corruption`` until it reaches a Poisson target length.
  Optional Zipf item popularity (rank ** -s over a seeded item permutation).
* ``dense_injected`` -- Bernoulli background plus item-disjoint injected
  patterns, each present in a transaction with its own probability.

Determinism: every draw comes from ``numpy.random.default_rng(seed)`` in a
fixed order, so the same numpy build gives bit-identical databases.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "n_words", "quest", "dense_injected", "uniform_random", "config", "batch_config",
    "batch_specs", "batch_one",
    "serve_pool", "serve_stream", "bitmap_to_csr", "CONFIG_SEED_BASE",
]

CONFIG_SEED_BASE = 10959


def n_words(m: int) -> int:
    """Number of u64 words per row for m items."""
    return (int(m) + 63) // 64


def _or_bits(rows: np.ndarray, r: np.ndarray, items: np.ndarray) -> None:
    """OR item bits into rows[r, items >> 6] (duplicates are harmless)."""
    if r.size == 0:
        return
    words = items >> 6
    bits = np.left_shift(np.uint64(1), (items & 63).astype(np.uint64))
    np.bitwise_or.at(rows, (r, words), bits)


def _pack_bool(b: np.ndarray, W: int) -> np.ndarray:
    """Pack a bool[c, m] matrix into uint64[c, W], item p at bit p&63 of word p>>6."""
    c, m = b.shape
    by = np.packbits(b, axis=1, bitorder="little")
    out = np.zeros((c, W * 8), np.uint8)
    out[:, : by.shape[1]] = by
    return out.view("<u8").astype(np.uint64, copy=False).reshape(c, W)


def quest(n: int, m: int, *, n_patterns: int, pat_len_mean: float, txn_len_mean: float,
          seed: int, zipf_s: float | None = None, corr_mean: float = 0.5,
          corr_sd: float = 0.1, max_draws: int = 64, chunk: int = 1 << 17):
    """Quest-style baskets.

    Returns (rows uint64[n, W], meta dict).  Patterns: length max(1, Poisson(
    pat_len_mean)) capped at m, items drawn without replacement with the item
    popularity; weights Exp(1) normalised; corruption N(corr_mean, corr_sd)
    clipped to [0, 1].  A transaction has target length max(1, Poisson(
    txn_len_mean)) and draws weighted patterns (each item kept with probability
    1 - corruption) until its distinct-item count reaches the target or
    ``max_draws`` draws were made.
    """
    rng = np.random.default_rng(seed)
    W = n_words(m)
    if zipf_s is None:
        p_item = np.full(m, 1.0 / m)
    else:
        perm = rng.permutation(m)
        w = np.arange(1, m + 1, dtype=np.float64) ** (-float(zipf_s))
        p_item = np.empty(m)
        p_item[perm] = w / w.sum()
    plen = np.minimum(np.maximum(1, rng.poisson(pat_len_mean, n_patterns)), m)
    lmax = int(plen.max())
    pat_items = np.full((n_patterns, lmax), -1, np.int64)
    for j in range(n_patterns):
        pat_items[j, : plen[j]] = rng.choice(m, size=int(plen[j]), replace=False, p=p_item)
    weights = rng.exponential(1.0, n_patterns)
    weights /= weights.sum()
    cdf = np.cumsum(weights)
    cdf[-1] = 1.0
    corr = np.clip(rng.normal(corr_mean, corr_sd, n_patterns), 0.0, 1.0)
    target = np.maximum(1, rng.poisson(txn_len_mean, n))
    rows = np.zeros((n, W), np.uint64)
    for start in range(0, n, chunk):
        stop = min(n, start + chunk)
        active = np.arange(start, stop)
        for _ in range(max_draws):
            if active.size == 0:
                break
            pj = np.minimum(np.searchsorted(cdf, rng.random(active.size), side="right"),
                            n_patterns - 1)
            items = pat_items[pj]
            keep = (rng.random(items.shape) >= corr[pj][:, None]) & (items >= 0)
            rr, cc = np.nonzero(keep)
            _or_bits(rows, active[rr], items[rr, cc])
            size = np.bitwise_count(rows[active]).sum(axis=1)
            active = active[size < target[active]]
    meta = {"generator": "quest", "n": n, "m": m, "n_patterns": n_patterns,
            "pat_len_mean": pat_len_mean, "txn_len_mean": txn_len_mean, "zipf_s": zipf_s,
            "corr_mean": corr_mean, "corr_sd": corr_sd, "seed": seed}
    return rows, meta


def dense_injected(n: int, m: int, *, background: float, pat_len_lo: int, pat_len_hi: int,
                   f_lo: float, f_hi: float, max_patterns: int, seed: int,
                   chunk: int = 1 << 16):
    """Bernoulli(background) on every (row, item), plus injected patterns.

    Patterns are item-disjoint: lengths U{pat_len_lo..pat_len_hi} are drawn and
    cut from a seeded item permutation until ``max_patterns`` are made or the
    next one no longer fits in m items.  Pattern j is present (all its items
    set) in each row independently with probability f_j ~ U[f_lo, f_hi].
    Returns (rows uint64[n, W], meta with the realised patterns).
    """
    rng = np.random.default_rng(seed)
    W = n_words(m)
    perm = rng.permutation(m)
    pats, pos = [], 0
    while len(pats) < max_patterns:
        ln = int(rng.integers(pat_len_lo, pat_len_hi + 1))
        if pos + ln > m:
            break
        pats.append(np.sort(perm[pos: pos + ln]))
        pos += ln
    f = rng.uniform(f_lo, f_hi, len(pats))
    pat_bool = np.zeros((len(pats), m), bool)
    for j, p in enumerate(pats):
        pat_bool[j, p] = True
    pat_words = _pack_bool(pat_bool, W) if pats else np.zeros((0, W), np.uint64)
    rows = np.zeros((n, W), np.uint64)
    for start in range(0, n, chunk):
        stop = min(n, start + chunk)
        c = stop - start
        blk = _pack_bool(rng.random((c, m)) < background, W)
        incl = rng.random((c, len(pats))) < f[None, :]
        for j in range(len(pats)):
            sel = incl[:, j]
            blk[sel] |= pat_words[j]
        rows[start:stop] = blk
    meta = {"generator": "dense_injected", "n": n, "m": m, "background": background,
            "patterns": [p.tolist() for p in pats], "f": f.tolist(), "seed": seed}
    return rows, meta


def uniform_random(n: int, m: int, density: float, seed: int):
    """Independent Bernoulli(density) bits; small test databases."""
    rng = np.random.default_rng(seed)
    return _pack_bool(rng.random((n, m)) < density, n_words(m))


def config(index: int, *, n: int | None = None):
    """The single-database workloads (index 1, 2, 3), seeded with 10959 + index.

    1: n=10,000, m=64, Quest-style, 200 patterns of mean length 4, transaction
       length mean 8; minsup 2 %, M = 1,000.
    2: n=1,000,000, m=1,000, Quest-style, 2,000 patterns of mean length 4,
       transaction length mean 10, Zipf(1.1) item popularity; minsup 0.5 %,
       M = 10,000.
    3: n=500,000, m=128, Bernoulli(0.35) background plus item-disjoint
       injected patterns of length 6..12, each in 20-40 % of the rows;
       minsup 30 %, M = 50,000.
    ``n`` overrides the row count (a prefix-sized instance of the same recipe).
    Returns dict(rows, m, minsup, M, name, meta).
    """
    seed = CONFIG_SEED_BASE + index
    if index == 1:
        nn = n or 10_000
        rows, meta = quest(nn, 64, n_patterns=200, pat_len_mean=4, txn_len_mean=8, seed=seed)
        return dict(name="quest_n10k_m64", rows=rows, m=64, minsup=0.02, M=1_000, meta=meta)
    if index == 2:
        nn = n or 1_000_000
        rows, meta = quest(nn, 1000, n_patterns=2000, pat_len_mean=4, txn_len_mean=10,
                           zipf_s=1.1, seed=seed)
        return dict(name="quest_zipf_n1M_m1000", rows=rows, m=1000, minsup=0.005, M=10_000,
                    meta=meta)
    if index == 3:
        nn = n or 500_000
        rows, meta = dense_injected(nn, 128, background=0.35, pat_len_lo=6, pat_len_hi=12,
                                    f_lo=0.2, f_hi=0.4, max_patterns=50, seed=seed)
        return dict(name="dense_n500k_m128", rows=rows, m=128, minsup=0.30, M=50_000, meta=meta)
    raise ValueError(f"no single-database config {index}")


def batch_config(count: int = 256, *, seed: int = CONFIG_SEED_BASE + 4,
                 n_lo: int = 1_000, n_hi: int = 200_000, widths=(64, 256, 1024),
                 len_lo: float = 8.0, len_hi: float = 20.0,
                 minsup_lo: float = 0.01, minsup_hi: float = 0.05, workers: int = 0):
    """Many independent Quest-style databases of uneven size and width.

    Per database: n ~ U{n_lo..n_hi}, m uniform from ``widths``, transaction
    length mean ~ U[len_lo, len_hi], 2*m latent patterns of mean length 4,
    minsup ~ U[minsup_lo, minsup_hi], M = max(1, n // 20).
    ``workers`` > 1 generates the databases in that many processes.
    Returns a list of dicts (rows, m, minsup, M, name, meta).
    """
    specs = batch_specs(count, seed=seed, n_lo=n_lo, n_hi=n_hi, widths=widths, len_lo=len_lo,
                        len_hi=len_hi, minsup_lo=minsup_lo, minsup_hi=minsup_hi)
    args = [(s["n"], s["m"], s["txn_len_mean"], s["subseed"]) for s in specs]
    mins = [s["minsup"] for s in specs]
    if workers > 1 and count > 1:
        # separate interpreters (spawned, never forked) so that a caller that
        # already holds a GPU context is not copied; same draws as serially
        import concurrent.futures as cf
        import multiprocessing as mp
        with cf.ProcessPoolExecutor(max_workers=min(workers, count),
                                    mp_context=mp.get_context("spawn")) as ex:
            made = list(ex.map(_batch_one, args, chunksize=4))
    else:
        made = [_batch_one(a) for a in args]
    out = []
    for i, (rows, meta) in enumerate(made):
        n, m = args[i][0], args[i][1]
        out.append(dict(name=f"batch{i}_n{n}_m{m}", rows=rows, m=m, minsup=float(mins[i]),
                        M=max(1, n // 20), meta=meta))
    return out


def batch_specs(count: int = 256, *, seed: int = CONFIG_SEED_BASE + 4,
                n_lo: int = 1_000, n_hi: int = 200_000, widths=(64, 256, 1024),
                len_lo: float = 8.0, len_hi: float = 20.0,
                minsup_lo: float = 0.01, minsup_hi: float = 0.05):
    """The draws of ``batch_config`` without generating any database: per
    database its n, m, transaction length mean, generator seed, minsup and M.
    ``batch_one(spec)`` makes database i's rows from its entry."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, count)
    ms = rng.choice(np.asarray(widths), count)
    lens = rng.uniform(len_lo, len_hi, count)
    mins = rng.uniform(minsup_lo, minsup_hi, count)
    subseeds = rng.integers(0, 2**31 - 1, count)
    return [dict(index=i, n=int(ns[i]), m=int(ms[i]), txn_len_mean=float(lens[i]),
                 subseed=int(subseeds[i]), minsup=float(mins[i]), M=max(1, int(ns[i]) // 20))
            for i in range(count)]


def batch_one(spec: dict):
    """Rows of one ``batch_specs`` entry (the same as ``batch_config``'s)."""
    return _batch_one((spec["n"], spec["m"], spec["txn_len_mean"], spec["subseed"]))[0]


def _batch_one(a):
    n, m, ln, sub = a
    return quest(n, m, n_patterns=2 * m, pat_len_mean=4, txn_len_mean=ln, seed=sub)


def serve_pool(*, seed: int = CONFIG_SEED_BASE + 5, n_small: int = 16, big_n_scale: float = 1.0):
    """Resident databases for the request stream: one of each single-database
    shape 2 and 3 (rows scaled by ``big_n_scale``) plus ``n_small`` batch-shaped
    databases.  Each entry carries the minsup range requests draw from:
    [0.5 %, 5 %] for the sparse shape, [25 %, 30 %] for the dense shape and
    [1 %, 5 %] for batch shapes."""
    pool = []
    c2 = config(2, n=int(1_000_000 * big_n_scale))
    c2["minsup_range"] = (0.005, 0.05)
    pool.append(c2)
    c3 = config(3, n=int(500_000 * big_n_scale))
    c3["minsup_range"] = (0.25, 0.30)
    pool.append(c3)
    for d in batch_config(n_small, seed=seed):
        d["minsup_range"] = (0.01, 0.05)
        pool.append(d)
    return pool


def serve_stream(pool_sizes, *, rate: float, duration_s: float, seed: int = CONFIG_SEED_BASE + 5,
                 minsup_ranges=None, big_share: float = 0.1):
    """Open-loop Poisson arrivals (mean ``rate`` per second) over ``duration_s``.

    Each request picks a database index (the first two, the large shapes, with
    total probability ``big_share``; the rest uniformly) and a minsup uniform in
    that database's range.  Returns a list of (t_arrival_s, db_index, minsup).
    """
    rng = np.random.default_rng(seed)
    ndb = len(pool_sizes)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration_s:
            break
        if ndb > 2 and rng.random() >= big_share:
            j = int(rng.integers(2, ndb))
        else:
            j = int(rng.integers(0, min(2, ndb)))
        lo, hi = minsup_ranges[j] if minsup_ranges else (0.01, 0.05)
        out.append((t, j, float(rng.uniform(lo, hi))))
    return out


def bitmap_to_csr(rows: np.ndarray, m: int):
    """Item lists of each row as CSR (items uint32, offsets uint64[n+1])."""
    n, W = rows.shape
    b = np.unpackbits(rows.astype("<u8").view(np.uint8).reshape(n, W * 8), axis=1,
                      bitorder="little")[:, :m]
    r, c = np.nonzero(b)
    offsets = np.zeros(n + 1, np.uint64)
    np.cumsum(np.bincount(r, minlength=n), out=offsets[1:])
    return c.astype(np.uint32), offsets
