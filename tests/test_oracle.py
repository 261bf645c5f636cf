"""Pins for the CPU oracle (no GPU).

Each test ties the oracle to something other than itself: hand-worked values,
the problem definition written out in pure Python, independent algorithms
(Apriori, exhaustive and tid-list enumeration), closed forms and invariants.
"""
import json
import os

import numpy as np
import pytest

import synth
from helpers import (apriori_gen, as_dict, is_canonical, items_of, np_support, pack,
                     py_bruteforce, unpack_bool)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
FIELDS = ("stop", "rows", "live", "promoted", "pruned", "generated", "solidified")


def _rand_db(seed, n, m, density):
    return synth.uniform_random(n, m, density, seed)


# ---------------------------------------------------------------- threshold

@pytest.mark.parametrize("minsup,n,tau", [
    (0.07, 100, 7),          # 0.07*100 = 7.000000000000001 in IEEE; the guard gives 7
    (0.02, 10_000, 200),
    (0.005, 1_000_000, 5_000),
    (0.30, 500_000, 150_000),
    (0.5, 6, 3),
    (0.5, 7, 4),             # 3.5 -> 4
    (1e-9, 1000, 1),         # never below 1
    (1.0, 10, 10),
    (1.5, 10, 11),           # unreachable threshold: n + 1
    (float("inf"), 10, 11),
])
def test_tau_pins(orc, minsup, n, tau):
    assert orc.tau(minsup, n) == tau


@pytest.mark.parametrize("minsup", [0.0, -0.1, float("nan")])
def test_tau_rejects(orc, minsup):
    with pytest.raises(orc.OracleError):
        orc.tau(minsup, 10)


# ---------------------------------------------------------------- subset test and first pass

def test_subset_test_exhaustive(orc):
    """(T AND I) == I against set inclusion for every I, T over 8 items."""
    rows = np.arange(256, dtype=np.uint64).reshape(256, 1)
    masks = np.arange(256, dtype=np.uint64).reshape(256, 1)
    got = orc.count_block(rows, 8, masks)
    want = np.array([sum(1 for t in range(256) if (set(items_of([t])) >= set(items_of([i]))))
                     for i in range(256)])
    assert np.array_equal(got, want)
    # one block at a time: every single row against every mask
    for t in (0, 1, 0x5A, 0xFF):
        got = orc.count_block(rows, 8, masks, first=t, last=t + 1)
        assert np.array_equal(got, np.array([int((i & t) == i) for i in range(256)]))


@pytest.mark.parametrize("m", [1, 63, 64, 65, 130, 1000])
def test_item_counts_vs_numpy(orc, m):
    rows = _rand_db(m, 300, m, 0.3)
    got = orc.item_counts(rows, m)
    want = unpack_bool(rows, m).sum(axis=0)
    assert np.array_equal(got, want)


def test_padding_bits_rejected(orc):
    rows = np.array([[1 << 10]], np.uint64)
    with pytest.raises(orc.OracleError):
        orc.dic(rows, 10, 0.5, 1)
    with pytest.raises(orc.OracleError):
        orc.dic(np.zeros((3, 1), np.uint64), 10, 0.5, 0)  # M = 0


# ---------------------------------------------------------------- hand-worked example

def test_hand_example():
    import oracle as orc
    g = json.load(open(os.path.join(GOLDEN, "hand_example.json")))
    rows = pack(g["rows"], g["m"])
    want = {tuple(items): c for items, c in g["frequent"]}
    assert orc.tau(g["minsup"], len(g["rows"])) == g["tau"]
    for run in g["runs"]:
        r = orc.dic(rows, g["m"], g["minsup"], run["M"])
        assert as_dict(r.masks, r.counts) == want
        assert is_canonical(r.masks)
        assert r.stats["stop_max"] == run["stop_max"]
        assert r.stats["stops"] == run["stops"]
        assert r.stats["tests"] == run["tests"]
        assert r.stats["peak_live"] == run["peak_live"]
        assert r.trace.tolist() == run["trace"], run["M"]
    for fn in (orc.apriori, orc.bruteforce, orc.tidlist):
        r = fn(rows, g["m"], g["minsup"])
        assert as_dict(r.masks, r.counts) == want


# ---------------------------------------------------------------- exhaustive cross-checks

CASES = [(s, n, m, d, ms) for s, (n, m, d, ms) in enumerate([
    (40, 6, 0.5, 0.2), (60, 8, 0.4, 0.1), (100, 10, 0.35, 0.05), (150, 12, 0.5, 0.15),
    (200, 16, 0.3, 0.04), (25, 5, 0.9, 0.5), (80, 14, 0.2, 0.01), (1, 7, 0.5, 0.5),
])]


@pytest.mark.parametrize("seed,n,m,density,minsup", CASES)
def test_bruteforce_vs_pure_python(orc, seed, n, m, density, minsup):
    rows = _rand_db(seed, n, m, density)
    lists = [items_of(r) for r in rows]
    want = py_bruteforce(lists, m, orc.tau(minsup, n))
    r = orc.bruteforce(rows, m, minsup)
    assert as_dict(r.masks, r.counts) == want
    assert is_canonical(r.masks)


@pytest.mark.parametrize("seed,n,m,density,minsup", CASES)
def test_dic_vs_bruteforce_all_M(orc, seed, n, m, density, minsup):
    rows = _rand_db(seed, n, m, density)
    want = as_dict(*_mc(orc.bruteforce(rows, m, minsup)))
    for M in sorted({1, 2, 3, 7, max(1, n // 2), max(1, n - 1), n, n + 1, 2 * n}):
        r = orc.dic(rows, m, minsup, M)
        assert as_dict(r.masks, r.counts) == want, M
        assert is_canonical(r.masks)
        assert r.stats["superset_prunes"] == 0
        assert r.stats["fullpass_promotions"] == 0
        if r.trace is not None:
            assert r.stats["tests"] == int((r.trace[:, 1] * r.trace[:, 2]).sum())
            assert r.stats["stops"] == len(r.trace)


def _mc(r):
    return r.masks, r.counts


@pytest.mark.parametrize("seed,n,m,density,minsup", [
    (11, 300, 64, 0.12, 0.03), (12, 200, 100, 0.08, 0.02), (13, 150, 130, 0.25, 0.12),
    (14, 400, 200, 0.03, 0.01),
])
def test_dic_vs_apriori_and_tidlist_wide(orc, seed, n, m, density, minsup):
    rows = _rand_db(seed, n, m, density)
    a = as_dict(*_mc(orc.apriori(rows, m, minsup)))
    t = as_dict(*_mc(orc.tidlist(rows, m, minsup)))
    assert a == t
    for M in (1, 17, n // 3, n):
        r = orc.dic(rows, m, minsup, M)
        assert as_dict(r.masks, r.counts) == a


def test_candgen_modes_identical_traces(orc):
    """New-box extension and the literal OR-of-all-box-pairs join agree stop by stop."""
    for seed, n, m, d, ms, M in [(21, 200, 12, 0.4, 0.08, 13), (22, 300, 16, 0.3, 0.03, 50),
                                 (23, 120, 10, 0.55, 0.2, 7), (24, 500, 64, 0.1, 0.01, 64)]:
        rows = _rand_db(seed, n, m, d)
        a = orc.dic(rows, m, ms, M, candgen_mode=0)
        b = orc.dic(rows, m, ms, M, candgen_mode=1)
        assert np.array_equal(a.masks, b.masks) and np.array_equal(a.counts, b.counts)
        assert np.array_equal(a.trace, b.trace)
        assert a.stats == b.stats


# ---------------------------------------------------------------- DIC-specific structure

def test_M_at_least_n_is_apriori(orc):
    """With one block per pass DIC is level-wise: the candidates counted at
    stop t are exactly apriori-gen of the frequent (t+1)-itemsets."""
    rows = _rand_db(31, 300, 14, 0.45)
    m, ms = 14, 0.06
    r = orc.dic(rows, m, ms, 300)
    L = as_dict(r.masks, r.counts)
    levels = {}
    for s in L:
        levels.setdefault(len(s), set()).add(s)
    assert r.stats["stop_max"] == 1
    for t, row in enumerate(r.trace):
        k = t + 1
        want = len(apriori_gen(levels.get(k, set())))
        assert int(row[2]) == want, (t, k)
        assert int(row[1]) == 300
    # the loop ends when a level produces no candidates
    assert len(apriori_gen(levels.get(len(r.trace) + 1, set()))) == 0


def test_prune_is_safe_and_work_accounting(orc):
    rows = _rand_db(41, 400, 12, 0.35)
    r = orc.dic(rows, 12, 0.05, 9)
    tr = r.trace
    assert r.stats["tests"] == int((tr[:, 1] * tr[:, 2]).sum())
    assert r.stats["peak_live"] == int(tr[:, 2].max())
    # live set evolves exactly by the recorded transitions
    for i in range(len(tr) - 1):
        assert tr[i + 1, 2] == tr[i, 2] - tr[i, 4] + tr[i, 5] - tr[i, 6]
    assert tr[-1, 2] - tr[-1, 4] + tr[-1, 5] - tr[-1, 6] == 0
    # rows per stop follow the block schedule with rewinding
    n, M = 400, 9
    smax = -(-n // M)
    for row in tr:
        s = int(row[0])
        assert 1 <= s <= smax
        assert int(row[1]) == min(s * M, n) - (s - 1) * M
    for i in range(len(tr) - 1):
        assert int(tr[i + 1, 0]) == int(tr[i, 0]) % smax + 1


# ---------------------------------------------------------------- closed forms

def test_closed_form_identical_rows(orc):
    T = [1, 4, 5, 9, 11]
    n = 37
    rows = pack([T] * n, 16)
    for M in (1, 5, 37, 100):
        r = orc.dic(rows, 16, 0.9, M)
        d = as_dict(r.masks, r.counts)
        assert len(d) == 2 ** len(T) - 1
        assert all(c == n for c in d.values())
        assert set(d) == {tuple(s) for k in range(1, 6)
                          for s in __import__("itertools").combinations(T, k)}


def test_closed_form_single_row(orc):
    T = [0, 3, 64, 100, 127]
    rows = pack([T], 128)
    r = orc.dic(rows, 128, 1.0, 1)
    assert len(r.counts) == 31 and set(r.counts.tolist()) == {1}


def test_closed_form_unreachable_threshold(orc):
    rows = _rand_db(51, 50, 20, 0.9)
    r = orc.dic(rows, 20, 1.01, 7)
    assert len(r.counts) == 0 and r.stats["stops"] == 0


def test_closed_form_disjoint_patterns(orc):
    """q disjoint patterns P_j, pattern j alone in r_j rows: L is every nonempty
    subset of each P_j with r_j >= tau, with count r_j."""
    pats = [[0, 1, 2], [5, 6], [10, 11, 12, 13], [20]]
    reps = [12, 4, 9, 30]
    lists = []
    for p, r in zip(pats, reps):
        lists += [p] * r
    n = len(lists)
    rows = pack(lists, 32)
    minsup = 9 / n
    tau = orc.tau(minsup, n)
    assert tau == 9
    import itertools
    want = {}
    for p, r in zip(pats, reps):
        if r >= tau:
            for k in range(1, len(p) + 1):
                for s in itertools.combinations(p, k):
                    want[s] = r
    for M in (1, 4, 11, n):
        r = orc.dic(rows, 32, minsup, M)
        assert as_dict(r.masks, r.counts) == want


def test_duplicated_database_doubles_counts(orc):
    rows = _rand_db(61, 200, 12, 0.4)
    a = orc.dic(rows, 12, 0.0731, 23)
    b = orc.dic(np.concatenate([rows, rows]), 12, 0.0731, 46)
    da, db = as_dict(a.masks, a.counts), as_dict(b.masks, b.counts)
    assert set(da) == set(db)
    assert all(db[s] == 2 * da[s] for s in da)


# ---------------------------------------------------------------- invariances

def test_transaction_permutation_invariance(orc):
    rows = _rand_db(71, 250, 40, 0.2)
    perm = np.random.default_rng(0).permutation(250)
    a = orc.dic(rows, 40, 0.03, 31)
    b = orc.dic(rows[perm], 40, 0.03, 31)
    assert as_dict(a.masks, a.counts) == as_dict(b.masks, b.counts)


def test_item_relabelling_equivariance(orc):
    m = 70
    rows = _rand_db(72, 200, m, 0.15)
    lists = [items_of(r) for r in rows]
    perm = np.random.default_rng(1).permutation(m)
    rows2 = pack([[int(perm[i]) for i in t] for t in lists], m)
    a = as_dict(*_mc(orc.dic(rows, m, 0.04, 19)))
    b = as_dict(*_mc(orc.dic(rows2, m, 0.04, 19)))
    mapped = {tuple(sorted(int(perm[i]) for i in s)): c for s, c in a.items()}
    assert mapped == b


def test_downward_closure_and_negative_border(orc):
    m = 24
    rows = _rand_db(81, 300, m, 0.3)
    r = orc.dic(rows, m, 0.05, 40)
    L = as_dict(r.masks, r.counts)
    tau = r.stats["tau"]
    for s, c in L.items():
        for x in range(len(s)):
            sub = s[:x] + s[x + 1:]
            if sub:
                assert sub in L and L[sub] >= c
    # negative border: itemsets not in L whose maximal subsets are all in L
    border = set()
    items = sorted({i for s in L for i in s})
    for s in L:
        for i in range(m):
            if i in s:
                continue
            c = tuple(sorted(s + (i,)))
            if c not in L and all(c[:x] + c[x + 1:] in L for x in range(len(c))):
                border.add(c)
    for i in range(m):
        if (i,) not in L:
            border.add((i,))
    sup = np_support(rows, m, sorted(border))
    assert (sup < tau).all()
    assert len(items) > 0


def test_counts_match_numpy_recount(orc):
    c = synth.config(1)
    r = orc.dic(c["rows"], c["m"], c["minsup"], c["M"])
    L = as_dict(r.masks, r.counts)
    keys = sorted(L)[:: max(1, len(L) // 150)]
    sup = np_support(c["rows"], c["m"], keys)
    assert sup.tolist() == [L[k] for k in keys]


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_openmp_build_matches_serial(orc, threads):
    """The OpenMP build of the same source (the timed CPU baseline) shares
    only the per-candidate count loop among threads: every result, statistic
    and trace entry equals the serial build's."""
    cases = [(synth.config(1), None)]
    for seed in (3, 11):
        rows = synth.uniform_random(1500, 70, 0.2, seed)
        cases.append(({"rows": rows, "m": 70, "minsup": 0.03, "M": 200}, seed))
    for c, _ in cases:
        ref = orc.dic(c["rows"], c["m"], c["minsup"], c["M"])
        got, used = orc.dic_parallel(c["rows"], c["m"], c["minsup"], c["M"], threads)
        assert used == threads
        assert np.array_equal(got.masks, ref.masks) and np.array_equal(got.counts, ref.counts)
        assert np.array_equal(got.trace, ref.trace)
        assert got.stats == ref.stats
