"""The row-to-item-bitset transposition at ragged shapes.

Every item's bitset feeds the first pass (its popcount is the item's
support) and every candidate's count (the AND of its items' bitsets), so a
bit moved to another item or another row changes a count.  With minsup low
enough that every item present is frequent (and pairs are counted), the
mined result must equal the oracle's at row counts around the 64-row word
and the 64-word tile, and widths around the 64-item word."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

SHAPES = [(1, 5, 0.6), (63, 64, 0.5), (64, 63, 0.5), (65, 65, 0.5), (4095, 130, 0.3),
          (4096, 64, 0.4), (4097, 300, 0.03), (4099, 1000, 0.02), (8193, 64, 0.5),
          (12295, 200, 0.1), (64 * 64 * 5 + 3, 129, 0.15)]


@pytest.mark.parametrize("n,m,d", SHAPES)
def test_transposed_bitsets_mine_like_the_oracle(n, m, d, orc):
    import paper_1812_10959_amd as dic
    rows = synth.uniform_random(n, m, d, 4000 + n % 997 + m)
    minsup = d * d * 0.9 if d >= 0.25 else d / 2
    if m >= 1000:  # every item frequent, no pair: keeps the oracle short
        minsup = 0.35 * d
    M = n // 3 + 1
    ref = orc.dic(rows, m, minsup, M)
    db = dic.dic_load_db(rows, m)
    r = dic.dic_mine(db, minsup, M)
    assert np.array_equal(r.masks, ref.masks) and np.array_equal(r.counts, ref.counts)
    assert np.array_equal(r.trace.astype(np.uint64), ref.trace)
