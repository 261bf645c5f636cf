"""GPU tests of the memory plumbing: a caller's allocator (torch's caching
allocator through ``use_torch``), an allocator that runs dry, and the
serving budget while a request's candidate pool overflows and restarts."""
import sys
import time

import numpy as np
import pytest

import synth
from helpers import pack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dic():
    import paper_1812_10959_amd as d
    yield d
    d.dic_set_allocator(None, None, None)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same(a, b):
    return (np.array_equal(a.masks, b.masks) and np.array_equal(a.counts, b.counts)
            and np.array_equal(a.trace, b.trace.astype(a.trace.dtype)))


def _equals_oracle(r, ref):
    return (np.array_equal(r.masks, ref.masks) and np.array_equal(r.counts, ref.counts)
            and np.array_equal(r.trace.astype(np.uint64), ref.trace))


def test_mine_through_torch_allocator_equals_oracle(dic, orc):
    """Database, candidate pools and rules all in torch's caching allocator;
    the result is the oracle's, from rows given as a host array and as a
    device tensor."""
    import torch
    c = synth.config(1)
    ref = orc.dic(c["rows"], c["m"], c["minsup"], c["M"])
    before = torch.cuda.memory_stats().get("allocation.all.allocated", 0)
    dic.use_torch()
    try:
        db = dic.dic_load_db(c["rows"], c["m"])
        r = dic.dic_mine(db, c["minsup"], c["M"])
        t = torch.from_numpy(c["rows"].view(np.int64)).cuda()
        db2 = dic.dic_load_db(t, c["m"])
        r2 = dic.dic_mine(db2, c["minsup"], c["M"])
        rb = dic.dic_batch([db, db2], [c["minsup"]] * 2, [c["M"]] * 2)
        after = torch.cuda.memory_stats().get("allocation.all.allocated", 0)
        dic.dic_free_db(db)
        dic.dic_free_db(db2)
    finally:
        dic.dic_set_allocator(None, None, None)
    _say(f"torch allocations made by the library: {after - before}")
    assert after - before >= 4  # two databases' rows and bitsets at least
    assert _equals_oracle(r, ref) and _equals_oracle(r2, ref)
    assert all(_equals_oracle(x, ref) for x in rb)


def test_allocator_running_dry_gives_nomem_and_no_leak(dic, orc):
    """An allocator that returns NULL after k blocks: the call fails with
    DIC_E_NOMEM, frees what it took (repeated failures do not accumulate
    blocks), and every block freed is one the allocator handed out."""
    import torch
    rows = synth.uniform_random(3000, 96, 0.12, 31)
    db = dic.dic_load_db(rows, 96)  # the library's own memory
    ref = orc.dic(rows, 96, 0.01, 400)
    live = {}
    stray = []
    limit = [0]
    made = [0]

    def alloc(size, _stream):
        if limit[0] <= 0:
            return None
        limit[0] -= 1
        made[0] += 1
        p = torch.cuda.caching_allocator_alloc(int(size))
        live[p] = size
        return p

    def free(p, _stream):
        if p not in live:
            stray.append(p)
            return
        del live[p]
        torch.cuda.caching_allocator_delete(p)

    dic.dic_set_allocator(alloc, free, None)
    try:
        # a first run with room: pooled engines keep their tables between
        # calls, so the blocks still held after a run are the baseline
        limit[0] = 1 << 30
        assert _equals_oracle(dic.dic_mine(db, 0.01, 400), ref)
        base = len(live)
        made[0] = 0
        assert _equals_oracle(dic.dic_mine(db, 0.01, 400), ref)
        per_run = made[0]  # blocks one run takes (its tables are pooled)
        assert per_run >= 2 and len(live) == base
        failures = 0
        for k in range(per_run):  # the (k+1)-th block is refused
            for _ in range(2):
                limit[0] = k
                with pytest.raises(dic.DicError) as e:
                    dic.dic_mine(db, 0.01, 400)
                assert e.value.code == dic.DIC_E_NOMEM, (k, e.value)
                failures += 1
                assert len(live) <= base, (k, len(live), base)
        limit[0] = 1 << 30
        assert _equals_oracle(dic.dic_mine(db, 0.01, 400), ref)
        assert len(live) <= base
    finally:
        dic.dic_set_allocator(None, None, None)
    assert not stray, f"{len(stray)} frees of blocks the allocator never made"
    _say(f"{failures} failures over {per_run} blocks per run, blocks held by pooled engines: "
         f"{len(live)} (baseline {base})")


def test_serve_budget_holds_through_overflow_restart(dic, orc):
    """16 items in every row: all 65,535 itemsets are frequent and the first
    candidate pool overflows.  Under a budget that fits the restarted request
    alone, the request gives its memory back, waits for the larger grant
    and then succeeds; other requests queue behind it.  The charge never
    exceeds the budget, and it reached the larger bound."""
    n, T = 6, list(range(16))
    rows = pack([T] * n, 16)
    db = dic.dic_load_db(rows, 16)
    big = dic.dic_serve_create(64 << 30)
    t = dic.dic_serve_submit(big, db, 0.5, 2)
    r = dic.dic_serve_wait(big, t, 60_000)
    _, peak_big, _ = dic.dic_serve_usage(big)
    dic.dic_serve_destroy(big)
    assert r.stats["restarts"] >= 1 and len(r.counts) == 2 ** 16 - 1
    # budgets doubling from 1 MiB: refused at submit, then admitted but
    # failing when the restarted pool's bound does not fit, then served
    outcomes, budget, peak1 = [], None, None
    for b in (1 << p for p in range(20, 36)):
        s = dic.dic_serve_create(b)
        try:
            tk = dic.dic_serve_submit(s, db, 0.5, 2)
        except dic.DicError as e:
            assert e.code == dic.DIC_E_CAPACITY
            outcomes.append("refused")
            dic.dic_serve_destroy(s)
            continue
        try:
            rr = dic.dic_serve_wait(s, tk, 60_000)
        except dic.DicError as e:
            assert e.code == dic.DIC_E_CAPACITY, e
            outcomes.append("outgrew")
            assert dic.dic_serve_usage(s)[1] <= b
            dic.dic_serve_destroy(s)
            continue
        used, peak1, bud = dic.dic_serve_usage(s)
        dic.dic_serve_destroy(s)
        assert _same(rr, r) and peak1 <= bud and used == 0
        outcomes.append("served")
        budget = b
        break
    _say(f"budgets from 1 MiB: {outcomes}; served at {budget}, peak {peak1} "
         f"(peak with a large budget {peak_big})")
    assert budget is not None and "outgrew" in outcomes
    assert peak1 == peak_big  # the same charges: the restart's bound included
    # several overflowing requests and small ones share that budget
    small_rows = synth.uniform_random(2000, 64, 0.1, 5)
    sdb = dic.dic_load_db(small_rows, 64)
    sref = dic.dic_mine(sdb, 0.02, 200)
    srv = dic.dic_serve_create(budget, max_active=8)
    tickets = []
    peaks = []
    for i in range(6):
        tickets.append(("big", dic.dic_serve_submit(srv, db, 0.5, 2)))
        tickets.append(("small", dic.dic_serve_submit(srv, sdb, 0.02, 200)))
        time.sleep(0.002)
        peaks.append(dic.dic_serve_usage(srv))
    for kind, tk in tickets:
        got = dic.dic_serve_wait(srv, tk, 120_000)
        assert _same(got, r if kind == "big" else sref), kind
        peaks.append(dic.dic_serve_usage(srv))
    used, peak, bud = dic.dic_serve_usage(srv)
    dic.dic_serve_destroy(srv)
    assert bud == budget and used == 0
    assert peak <= budget and all(u <= budget for u, _, _ in peaks)
    assert peak >= peak1
    ref = orc.dic(rows, 16, 0.5, 2)
    assert _equals_oracle(r, ref)


def test_serve_charges_resident_database(dic):
    """A database's rows and bitsets count once against the budget while
    requests on it are admitted, and not after."""
    rows = synth.uniform_random(50_000, 1024, 0.01, 8)
    db = dic.dic_load_db(rows, 1024)
    db_bytes = rows.nbytes + 1024 * ((50_000 + 63) // 64) * 8
    srv = dic.dic_serve_create(64 << 30, max_active=4)
    ts = [dic.dic_serve_submit(srv, db, 0.05, 5000) for _ in range(3)]
    seen = [dic.dic_serve_usage(srv)[0]]
    for t in ts:
        dic.dic_serve_wait(srv, t, 60_000)
    used, peak, _ = dic.dic_serve_usage(srv)
    dic.dic_serve_destroy(srv)
    assert used == 0 and peak >= db_bytes and max(seen) <= peak
    # one request's bound plus the database exceeds a budget of the bound alone
    one = dic.dic_serve_create(64 << 30, max_active=1)
    t = dic.dic_serve_submit(one, db, 0.05, 5000)
    dic.dic_serve_wait(one, t, 60_000)
    _, peak1, _ = dic.dic_serve_usage(one)
    dic.dic_serve_destroy(one)
    tight = dic.dic_serve_create(peak1 - db_bytes // 2)
    with pytest.raises(dic.DicError) as e:
        dic.dic_serve_submit(tight, db, 0.05, 5000)
    assert e.value.code == dic.DIC_E_CAPACITY
    dic.dic_serve_destroy(tight)
