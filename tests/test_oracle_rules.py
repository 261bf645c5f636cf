"""Pins of the oracle's association-rule generation (CPU only).

The oracle derives rules from a frequent-itemset result.  It is pinned to
things other than itself: a hand-worked example, a brute force that counts
every antecedent directly in the transactions, closed forms and invariants
of the definition.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle as orc

from helpers import items_of, pack

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rules_hand_example.json")


def _rule_set(res, R):
    """{(antecedent items, consequent items): (supp_I, supp_X)} from oracle rules."""
    out = {}
    for i, code, sx in zip(R.itemset, R.code, R.supp_x):
        I = items_of(res.masks[i])
        X = tuple(I[t] for t in range(len(I)) if (int(code) >> t) & 1)
        Y = tuple(x for x in I if x not in X)
        out[(X, Y)] = (int(res.counts[i]), int(sx))
    return out


def test_hand_example():
    g = json.load(open(GOLDEN))
    names = g["items"]
    idx = {c: i for i, c in enumerate(names)}
    rows = pack([[idx[c] for c in t] for t in g["transactions"]], len(names))
    res = orc.bruteforce(rows, len(names), g["minsup"])
    got_freq = {"".join(names[i] for i in items_of(mk)): int(c)
                for mk, c in zip(res.masks, res.counts)}
    assert got_freq == g["frequent"]
    for case in g["cases"]:
        R = orc.rules(res.masks, res.counts, case["minconf"])
        got = {("".join(names[i] for i in X), "".join(names[i] for i in Y))
               for (X, Y) in _rule_set(res, R)}
        assert got == {tuple(r) for r in case["rules"]}, case["note"]


def _brute_rules(rows, res, minconf):
    """Rules by definition, counting every antecedent in the transactions."""
    W = rows.shape[1]
    out = []
    for i, (mk, cI) in enumerate(zip(res.masks, res.counts)):
        I = items_of(mk)
        k = len(I)
        if k < 2:
            continue
        for code in range(1, (1 << k) - 1):
            X = [I[t] for t in range(k) if (code >> t) & 1]
            xm = np.zeros(W, np.uint64)
            for p in X:
                xm[p >> 6] |= np.uint64(1) << np.uint64(p & 63)
            sx = int(((rows & xm) == xm).all(axis=1).sum())
            if float(cI) >= minconf * float(sx):
                out.append((i, code, sx))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_against_brute_force(seed):
    rng = np.random.default_rng(900 + seed)
    n, m = int(rng.integers(20, 200)), int(rng.integers(3, 11))
    dens = rng.uniform(0.2, 0.6)
    rows = pack([[i for i in range(m) if rng.random() < dens] for _ in range(n)], m)
    res = orc.bruteforce(rows, m, float(rng.uniform(0.05, 0.3)))
    for minconf in (0.0, 0.3, 0.5, 0.8, 1.0):
        R = orc.rules(res.masks, res.counts, minconf)
        got = list(zip(R.itemset.tolist(), R.code.tolist(), R.supp_x.tolist()))
        assert got == _brute_rules(rows, res, minconf), (seed, minconf)


@pytest.mark.parametrize("t", [2, 3, 5, 8])
def test_identical_transactions_closed_form(t):
    # every subset of T is frequent with count n, so every rule has confidence 1:
    # sum_{k>=2} C(t,k) (2^k - 2) = 3^t - 2^(t+1) + 1 rules for any minconf <= 1
    m = 12
    T = list(range(1, 1 + t))
    rows = pack([T] * 7, m)
    res = orc.bruteforce(rows, m, 0.5)
    assert len(res.counts) == 2 ** t - 1
    for minconf in (0.0, 0.5, 1.0):
        R = orc.rules(res.masks, res.counts, minconf)
        assert len(R.itemset) == 3 ** t - 2 ** (t + 1) + 1
        assert (R.supp_x == 7).all()
    assert len(orc.rules(res.masks, res.counts, 1.0000001).itemset) == 0


def test_zero_minconf_keeps_every_split_and_confidence_monotone():
    rng = np.random.default_rng(5)
    m = 9
    rows = pack([[i for i in range(m) if rng.random() < 0.5] for _ in range(150)], m)
    res = orc.bruteforce(rows, m, 0.1)
    ks = [len(items_of(mk)) for mk in res.masks]
    R = orc.rules(res.masks, res.counts, 0.0)
    assert len(R.itemset) == sum(2 ** k - 2 for k in ks if k >= 2)
    # for a fixed I, confidence can only grow as the antecedent grows
    # (supp is anti-monotone), so the kept antecedents are closed upwards
    for minconf in (0.4, 0.7):
        Rc = orc.rules(res.masks, res.counts, minconf)
        kept = {}
        for i, code in zip(Rc.itemset.tolist(), Rc.code.tolist()):
            kept.setdefault(i, set()).add(code)
        for i, codes in kept.items():
            full = (1 << ks[i]) - 1
            for c in codes:
                for t in range(ks[i]):
                    sup = c | (1 << t)
                    if sup != c and sup != full:
                        assert sup in codes, (i, c, sup)


def test_errors():
    # a frequent pair whose singleton is missing: not downward closed
    masks = np.array([[0b1], [0b11]], np.uint64)
    with pytest.raises(orc.OracleError) as e:
        orc.rules(masks, np.array([5, 3], np.uint32), 0.5)
    assert e.value.code == orc.OR_E_INVAL
    big = np.array([[(1 << 25) - 1]], np.uint64)
    with pytest.raises(orc.OracleError) as e:
        orc.rules(big, np.array([3], np.uint32), 0.5)
    assert e.value.code == orc.OR_E_RANGE
    assert len(orc.rules(np.zeros((0, 1), np.uint64), np.zeros(0, np.uint32), 0.5).itemset) == 0
