#!/usr/bin/env python3
"""Benchmark: frequent itemset mining by Dynamic Itemset Counting on one MI355X.

A step is one full mining call (first pass, then every stop: count, prune /
promote, candidate generation, full-pass check and compaction, then
collection) over the sparse Quest-style database of n = 1,000,000
transactions and m = 1,000 items (minsup 0.5 %, M = 10,000), resident in HBM
before timing starts.  ``value`` is subset tests per second over the whole
step: (sum over stops of live candidates x block rows, plus the m*n item tests
of the first pass) / step time.

Also reported on the same line: the count kernel's roofline (HIP-event time
of every CountSupport launch, algorithmic work per launch), the CPU oracle on
a bounded sample, the other single-database workloads, batched vs plain
mining of 256 databases, and latency percentiles of a served Poisson request
stream.  Progress goes to stderr; the JSON line to stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "G subset-tests/s & % HBM roofline, batched vs plain; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz: 32-bit integer VALU lane operations
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--only-headline", action="store_true",
                    help="time the headline workload only (for profiler runs)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--cpu-rows", type=int, default=40_000)
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the parallel CPU oracle on the whole headline workload "
                         "(0: min(16, CPUs available); -1: skip it)")
    ap.add_argument("--no-layouts", action="store_true",
                    help="skip the profiled count-kernel passes (for counter runs)")
    ap.add_argument("--layouts", default="1,0",
                    help="counting layouts of the profiled passes (1 item bitsets, 0 rows)")
    ap.add_argument("--layout", type=int, default=1, choices=(0, 1),
                    help="counting layout of the timed headline steps (default 1)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also copy the headline rows device to device once (a copy of known "
                         "size for scaling memory counters)")
    return ap.parse_args()


def mine_rate(stats, n, m):
    return (stats["tests"] + n * m)


def count_work(results, W, n_frequent_items, layout):
    """Algorithmic work of the CountSupport launches of these results.

    Per stop s with B_s block rows, K_s live candidates, sum of their sizes
    I_s and nonzero 32-bit mask words Z_s:
      item bitsets (layout 1): bytes = F * ceil(B_s/64) * 8 (the frequent
        items' words of the block, read once) + K_s * 16 (mask word, count);
        lane-ops = 2 * I_s * ceil(B_s/64) (one 64-bit AND per item beyond
        the first and one 64-bit popcount per candidate and word, two 32-bit
        lane operations each);
      row bitmaps (layout 0): bytes = B_s * 8W + K_s * 8W; lane-ops =
        (Z_s + K_s) * B_s (one AND-accumulate per nonzero word and one
        compare per candidate and row)."""
    byt = ops = 0.0
    ms = 0.0
    launches = 0
    for r in results:
        rows = r.trace[:, 1].astype(np.float64)
        live = r.trace[:, 2].astype(np.float64)
        if layout == 1:
            words64 = np.ceil(rows / 64.0)
            byt += float((n_frequent_items * words64 * 8 + live * 16).sum())
            ops += float((2.0 * r.items.astype(np.float64) * words64).sum())
        else:
            byt += float((rows * 8 * W + live * 8 * W).sum())
            ops += float(((r.words.astype(np.float64) + live) * rows).sum())
        ms += r.stats["count_ms"]
        launches += r.stats["count_launches"]
    return byt, ops, ms, launches


PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_stop_quest_zipf_n1M_m1000_pmc.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1812_10959_amd", "csrc", "dic_kernels.hip")


def measured_traffic():
    """HBM bytes per k_stop launch from the committed rocprofv3 counter
    runs (FETCH_SIZE and WRITE_SIZE scaled by a copy of known size), or None
    when the kernel source changed since the counters were taken."""
    import hashlib
    try:
        txt = open(PMC_SUMMARY).read()
    except OSError:
        return None
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if sha not in txt:
        return None
    for ln in txt.splitlines():
        if ln.startswith("k_stop traffic_bytes_per_launch:"):
            return float(ln.split(":")[1])
    return None


def roofline_entry(byt, ops, ms, launches):
    achieved_tops = ops / (ms * 1e-3) / 1e12 if ms else 0.0
    achieved_gbs = byt / (ms * 1e-3) / 1e9 if ms else 0.0
    return {
        "kernel": "k_stop", "bound": "alu", "achieved": achieved_tops,
        "peak": ALU_PEAK_TOPS, "unit": "Tops/s (int32 VALU lane-ops)",
        "frac": achieved_tops / ALU_PEAK_TOPS, "traffic": None,
        "hbm": {"achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved_gbs / HBM_PEAK_GBS},
        "avg_launch_us": ms / launches * 1e3 if launches else 0.0,
        "launches": launches, "count_ms": ms,
        "algorithmic_bytes_per_launch": byt / launches if launches else 0.0,
    }


def headline(dic, args, c):
    rows, m = c["rows"], c["m"]
    n, W = rows.shape
    db = dic.dic_load_db(rows, m)
    dic.dic_set_option("profile", 0)
    dic.dic_set_option("layout", args.layout)
    import torch
    for i in range(args.warmup):
        r = dic.dic_mine(db, c["minsup"], c["M"])
        log(f"  warmup {i}: {r.stats['mine_ms']:.1f} ms, |L|={r.stats['n_frequent']}, "
            f"stops={r.stats['stops']}")
    torch.cuda.synchronize()
    res = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        res.append(dic.dic_mine(db, c["minsup"], c["M"]))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for r in res[1:]:
        assert np.array_equal(r.masks, res[0].masks) and np.array_equal(r.counts, res[0].counts)
    st = res[0].stats
    tests = mine_rate(st, n, m)
    value = tests * args.steps / dt / 1e9
    log(f"  timed {args.steps} steps: {dt / args.steps * 1e3:.2f} ms/step, {value:.1f} G tests/s")
    out = {"value": value, "ms_per_step": dt / args.steps * 1e3, "stats": st,
           "workload": c, "db": db, "rows": rows, "result": res[0]}
    if args.calibrate_copy:
        t = torch.from_numpy(rows.view(np.int64)).cuda()
        torch.cuda.synchronize()
        dic.dic_load_db(t, m)  # one device-to-device copy of n*W*8 bytes
        log(f"  calibration copy: {rows.nbytes} bytes device to device")
    # Count-kernel roofline: a second timed region with HIP events around
    # every CountSupport launch (profiled runs launch directly, not as graphs).
    n_freq_items = int((np.bitwise_count(res[0].masks).sum(axis=1) == 1).sum())
    layouts = {}
    first_pass = {}
    for layout in (() if args.no_layouts else [int(x) for x in args.layouts.split(",") if x]):
        dic.dic_set_option("layout", layout)
        dic.dic_set_option("profile", 1)
        prof = []
        reps = args.steps if layout == 1 else max(1, min(2, args.steps))
        t0 = time.perf_counter()
        for _ in range(reps):
            prof.append(dic.dic_mine(db, c["minsup"], c["M"]))
        pdt = (time.perf_counter() - t0) / reps
        dic.dic_set_option("profile", 0)
        byt, ops, cms, launches = count_work(prof, W, n_freq_items, layout)
        entry = roofline_entry(byt, ops, cms, launches)
        # the timed launches: k_stop (one stop: MakeCandidates, CountSupport
        # and Prune of new and surviving candidates, then the serial part);
        # with row bitmaps k_count runs first, between the same events
        entry["kernel"] = "k_stop" if layout == 1 else "k_count + k_stop"
        entry["count_ms_per_step"] = cms / reps
        entry["mine_ms_per_step_profiled"] = pdt * 1e3
        entry["count_G_tests_per_s"] = st["tests"] / (cms / reps * 1e-3) / 1e9 if cms else 0.0
        entry["bytes_per_step"] = byt / reps
        entry["ops_per_step"] = ops / reps
        layouts["item_bitsets" if layout == 1 else "row_bitmaps"] = entry
        log(f"  layout {layout}: count {cms / reps:.2f} ms/step over {launches // reps} launches,"
            f" {entry['achieved']:.3f} Tops/s ({100 * entry['frac']:.2f}% ALU), "
            f"{entry['hbm']['achieved']:.1f} GB/s, mine {pdt * 1e3:.1f} ms profiled")
        first_pass[layout] = [r.stats["first_pass_ms"] for r in prof]
    if first_pass:
        out["first_pass"] = first_pass_entry(dic, db, c, first_pass, args.steps)
    dic.dic_set_option("layout", 1)
    if "item_bitsets" in layouts:
        layouts["item_bitsets"]["traffic"] = measured_traffic()
        layouts["item_bitsets"]["traffic_unit"] = "bytes per launch (HBM, rocprofv3 counters)"
    out["roofline"] = layouts.get("item_bitsets")
    out["layouts"] = layouts
    return out


def _flush_caches(torch, buf):
    """Evict the L2s and the 256 MB Infinity Cache: write 1 GiB."""
    buf.fill_(1)
    torch.cuda.synchronize()


def first_pass_entry(dic, db, c, warm, reps):
    """FirstPass against the HBM roof: every item's bitset (m * ceil(n/64)
    words) or every row (n * W words) is read once per mine.  Warm: the
    profiled mines above, the database resident in the Infinity Cache from
    the previous mine.  Cold: each mine after 1 GiB of writes."""
    import torch
    rows = c["rows"]
    n, W = rows.shape
    m = c["m"]
    nw = (n + 63) // 64
    buf = torch.empty(1 << 27, dtype=torch.int64, device="cuda")
    out = {}
    for layout, name, byt, kernel in ((1, "item_bitsets", m * nw * 8, "k_first_pass_vert"),
                                      (0, "row_bitmaps", n * W * 8, "k_first_pass")):
        if layout not in warm:
            continue
        dic.dic_set_option("layout", layout)
        dic.dic_set_option("profile", 1)
        cold = []
        for _ in range(max(3, min(reps, 5)) if layout == 1 else 2):
            _flush_caches(torch, buf)
            cold.append(dic.dic_mine(db, c["minsup"], c["M"]).stats["first_pass_ms"])
        dic.dic_set_option("profile", 0)
        w_ms, c_ms = float(np.median(warm[layout])), float(np.median(cold))
        e = {"kernel": kernel, "bound": "hbm", "algorithmic_bytes_per_launch": byt,
             "unit": "GB/s", "peak": HBM_PEAK_GBS,
             "cold": {"ms": c_ms, "achieved": byt / (c_ms * 1e-3) / 1e9,
                      "frac": byt / (c_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "runs": len(cold)},
             "warm": {"ms": w_ms, "achieved": byt / (w_ms * 1e-3) / 1e9,
                      "frac": byt / (w_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "runs": len(warm[layout])}}
        out[name] = e
        log(f"  first pass ({name}): cold {c_ms * 1e3:.1f} us = {e['cold']['achieved']:.0f} GB/s "
            f"({100 * e['cold']['frac']:.1f}% HBM), warm {w_ms * 1e3:.1f} us = "
            f"{e['warm']['achieved']:.0f} GB/s")
    del buf
    return out


def load_entry(dic, c):
    """dic_load_db from rows already on the device: one device copy of the
    rows (n * W words read and written), the padding check (read) and the
    transposition into item bitsets (rows read, m * ceil(n/64) words
    written)."""
    import torch
    rows = c["rows"]
    n, W = rows.shape
    nw = (n + 63) // 64
    t = torch.from_numpy(rows.view(np.int64)).cuda()
    torch.cuda.synchronize()
    dic.dic_free_db(dic.dic_load_db(t, c["m"]))
    times = []
    for _ in range(5):
        t0 = time.perf_counter()
        db = dic.dic_load_db(t, c["m"])
        times.append(time.perf_counter() - t0)
        dic.dic_free_db(db)
    ms = float(np.median(times)) * 1e3
    byt = 4 * n * W * 8 + c["m"] * nw * 8
    log(f"  load from device rows: {ms:.3f} ms ({byt / (ms * 1e-3) / 1e9:.0f} GB/s of copy, "
        "check and transposition bytes)")
    return {"ms": ms, "bytes": byt, "GB_per_s": byt / (ms * 1e-3) / 1e9,
            "note": "wall time of dic_load_db on a device tensor: copy + padding check + "
                    "k_transpose; the kernel alone is in the committed rocprofv3 trace"}


def cpu_baseline(c, rows_full, n_rows, threads, gpu_result):
    """The CPU oracle timed two ways on the host: the serial checker (-O2, one
    thread) on a prefix of the headline rows, and the same source built -O3
    -march=native -fopenmp, its count loop over the live candidates shared
    among `threads` threads, on the whole headline workload (its result is
    compared with the GPU's)."""
    import oracle
    rows = np.ascontiguousarray(rows_full[:n_rows])
    log(f"CPU oracle on the first {n_rows} rows ...")
    t0 = time.perf_counter()
    r = oracle.dic(rows, c["m"], c["minsup"], c["M"])
    dt = time.perf_counter() - t0
    tests = r.stats["tests"] + n_rows * c["m"]
    log(f"  oracle {dt:.1f}s, {tests / dt / 1e9:.3f} G tests/s")
    out = {"value": tests / dt / 1e9, "unit": "G subset-tests/s", "cores": 1, "kind": "oracle",
           "sample": f"first {n_rows} rows of the n=1,000,000 m=1,000 workload, same minsup and "
                     f"M (stop_max {r.stats['stop_max']}, not 100); serial C oracle built -O2, "
                     f"{dt:.1f} s, {r.stats['tests']} block tests + {n_rows * c['m']} first-pass "
                     "tests",
           "cpu": _cpu_model(), "host_cpus": _host_cpus()}
    if threads > 0:
        n, m = rows_full.shape[0], c["m"]
        log(f"CPU oracle, OpenMP build, {threads} threads, whole workload ...")
        t0 = time.perf_counter()
        rp, used = oracle.dic_parallel(rows_full, m, c["minsup"], c["M"], threads)
        dtp = time.perf_counter() - t0
        tp = rp.stats["tests"] + n * m
        same = (np.array_equal(rp.masks, gpu_result.masks)
                and np.array_equal(rp.counts, gpu_result.counts)
                and np.array_equal(rp.trace, gpu_result.trace.astype(rp.trace.dtype)))
        log(f"  oracle (OpenMP) {dtp:.1f}s on {used} threads, {tp / dtp / 1e9:.3f} G tests/s, "
            f"equal to the GPU result: {same}")
        out["parallel"] = {
            "value": tp / dtp / 1e9, "unit": "G subset-tests/s", "cores": used,
            "kind": "oracle, parallel count loop",
            "sample": f"the whole n={n:,} m={m:,} workload (minsup {c['minsup']}, M {c['M']}); "
                      "oracle source built -O3 -march=native -fopenmp, the count over live "
                      f"candidates shared by {used} threads, {dtp:.1f} s",
            "seconds": dtp, "threads": used, "cpu": _cpu_model(), "host_cpus": _host_cpus(),
            "identical_to_gpu_result": bool(same)}
    return out


def _host_cpus():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count()


def _cpu_model():
    """The host CPU as /proc/cpuinfo names it, with its family, model and
    stepping numbers (a virtual machine may show a short model name)."""
    info = {}
    try:
        for ln in open("/proc/cpuinfo"):
            if ":" in ln:
                k, v = (x.strip() for x in ln.split(":", 1))
                if k in ("model name", "cpu family", "model", "stepping") and k not in info:
                    info[k] = v
            elif info:
                break
    except OSError:
        return "unknown"
    return (f"{info.get('model name', 'unknown')} (family {info.get('cpu family', '?')}, "
            f"model {info.get('model', '?')}, stepping {info.get('stepping', '?')})")


def other_configs(dic, inputs):
    out = {}
    for c in inputs:
        rows, m = c["rows"], c["m"]
        n = rows.shape[0]
        db = dic.dic_load_db(rows, m)
        for _ in range(2):
            dic.dic_mine(db, c["minsup"], c["M"])
        times = []
        for _ in range(7):  # median of seven: one slow call does not move it
            t0 = time.perf_counter()
            r = dic.dic_mine(db, c["minsup"], c["M"])
            times.append(time.perf_counter() - t0)
        dt = float(np.median(times))
        st = r.stats
        out[c["name"]] = {
            "n": n, "m": m, "minsup": c["minsup"], "M": c["M"], "ms": dt * 1e3,
            "G_tests_per_s": mine_rate(st, n, m) / dt / 1e9,
            "count_G_tests_per_s": st["tests"] / (st["count_ms"] * 1e-3) / 1e9
            if st["count_ms"] else None,
            "n_frequent": st["n_frequent"], "k_max": st["k_max"], "stops": st["stops"],
            "tests": st["tests"], "peak_live": st["peak_live"]}
        log(f"  {c['name']}: {dt * 1e3:.2f} ms, {out[c['name']]['G_tests_per_s']:.1f} G tests/s")
    return out


def rules_bench(dic, cases, minconf=0.5):
    """Association rules from mining results: device time of the two passes,
    whole-call time, and the oracle's time on the same itemsets."""
    import oracle
    out = {}
    for name, db, c in cases:
        res = dic.dic_mine(db, c["minsup"], c["M"])
        dic.dic_rules(res, minconf)
        runs = [dic.dic_rules(res, minconf) for _ in range(5)]
        k_ms = float(np.median([r.stats["kernel_ms"] for r in runs]))
        t_ms = float(np.median([r.stats["total_ms"] for r in runs]))
        st = runs[0].stats
        t0 = time.perf_counter()
        ref = oracle.rules(res.masks, res.counts, minconf)
        o_s = time.perf_counter() - t0
        assert len(ref.itemset) == st["rules"]
        out[name] = {"minconf": minconf, "itemsets": int(st["itemsets"]),
                     "splits": int(st["splits"]), "rules": int(st["rules"]),
                     "kernel_ms": k_ms, "total_ms": t_ms,
                     "G_splits_per_s_kernel": st["splits"] / (k_ms * 1e-3) / 1e9 if k_ms else None,
                     "oracle_s": o_s, "oracle_cores": 1}
        log(f"  rules {name}: {st['splits']} splits, {st['rules']} rules, kernel {k_ms:.3f} ms, "
            f"call {t_ms:.2f} ms, oracle {o_s:.2f} s")
    return out


def batch_vs_plain(dic, dbs_spec):
    count = len(dbs_spec)
    dbs = [dic.dic_load_db(d["rows"], d["m"]) for d in dbs_spec]
    ms = [d["minsup"] for d in dbs_spec]
    Ms = [d["M"] for d in dbs_spec]
    tests_first = sum(d["rows"].shape[0] * d["m"] for d in dbs_spec)
    # warm both paths once
    dic.dic_batch(dbs[:8], ms[:8], Ms[:8])
    for i in range(4):
        dic.dic_mine(dbs[i], ms[i], Ms[i])
    t0 = time.perf_counter()
    plain = [dic.dic_mine(db, a, b) for db, a, b in zip(dbs, ms, Ms)]
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    batched = dic.dic_batch(dbs, ms, Ms)
    t_batch = time.perf_counter() - t0
    same = all(np.array_equal(p.masks, b.masks) and np.array_equal(p.counts, b.counts)
               for p, b in zip(plain, batched))
    tests = sum(r.stats["tests"] for r in plain) + tests_first
    out = {"databases": count, "plain_s": t_plain, "batched_s": t_batch,
           "plain_G_tests_per_s": tests / t_plain / 1e9,
           "batched_G_tests_per_s": tests / t_batch / 1e9,
           "speedup": t_plain / t_batch, "identical_results": bool(same),
           "total_tests": tests,
           "n_frequent_total": int(sum(r.stats["n_frequent"] for r in plain))}
    log(f"  plain {t_plain:.2f}s, batched {t_batch:.2f}s, x{t_plain / t_batch:.2f}, "
        f"identical={same}")
    return out


def _serve_run(dic, pool, dbs, rate, seconds, seed=None):
    """Open-loop Poisson arrivals at `rate` for `seconds` on a fresh server."""
    import synth
    kw = {} if seed is None else {"seed": seed}
    stream = synth.serve_stream([p["rows"].shape[0] for p in pool], rate=rate,
                                duration_s=seconds, minsup_ranges=[p["minsup_range"] for p in pool],
                                **kw)
    srv = dic.dic_serve_create(200 << 30, max_active=64)
    tickets = []
    t_start = time.perf_counter()
    for (t_arr, j, minsup) in stream:
        now = time.perf_counter() - t_start
        if t_arr > now:
            time.sleep(t_arr - now)
        M = pool[j]["M"] if j < 2 else max(1, pool[j]["rows"].shape[0] // 20)
        tickets.append((dic.dic_serve_submit(srv, dbs[j], minsup, M), j, minsup, M))
    results = []
    for (t, j, minsup, M) in tickets:
        results.append((dic.dic_serve_wait(srv, t), j, minsup, M))
    wall = time.perf_counter() - t_start
    p50, p99, rps = dic.dic_serve_stats(srv)
    dic.dic_serve_destroy(srv)
    return results, wall, p50, p99, rps


def serving(dic, seconds, rate, c2, c3, small):
    log(f"serving: Poisson {rate}/s for {seconds}s over mixed databases ...")
    pool = [dict(c2, minsup_range=(0.005, 0.05)), dict(c3, minsup_range=(0.25, 0.30))]
    for d in small:
        pool.append(dict(d, minsup_range=(0.01, 0.05)))
    dbs = [dic.dic_load_db(p["rows"], p["m"]) for p in pool]
    results, wall, p50, p99, rps = _serve_run(dic, pool, dbs, rate, seconds)
    log(f"  {len(results)} requests served")
    # spot-check that served results equal solo mining
    rng = np.random.default_rng(0)
    ok = True
    for k in rng.choice(len(results), size=min(8, len(results)), replace=False):
        r, j, minsup, M = results[k]
        solo = dic.dic_mine(dbs[j], minsup, M)
        ok &= np.array_equal(r.masks, solo.masks) and np.array_equal(r.counts, solo.counts)
    tests = sum(r.stats["tests"] + pool[j]["rows"].shape[0] * pool[j]["m"]
                for r, j, _, _ in results)
    out = {"rate_req_per_s": rate, "seconds": seconds, "requests": len(results),
           "p50_ms": p50, "p99_ms": p99, "throughput_req_per_s": rps,
           "G_tests_per_s": tests / wall / 1e9, "budget_bytes": 200 << 30,
           "spot_check_identical": bool(ok)}
    log(f"  p50 {p50:.1f} ms, p99 {p99:.1f} ms, {rps:.1f} req/s, spot-check identical={ok}")
    # sustainable rate: offered rates doubled until the server falls behind
    # (completions below 95 % of the offered rate or p99 above 250 ms)
    sweep, best = [], None
    r = 2 * rate
    while r <= 32 * rate:
        res, w, a50, a99, arps = _serve_run(dic, pool, dbs, r, 3.0, seed=int(r))
        kept = arps >= 0.95 * r and a99 <= 250.0
        sweep.append({"rate_req_per_s": r, "requests": len(res), "p50_ms": a50, "p99_ms": a99,
                      "throughput_req_per_s": arps, "keeps_up": bool(kept)})
        log(f"  offered {r:.0f}/s: {arps:.0f} req/s done, p50 {a50:.1f} ms, p99 {a99:.1f} ms")
        if not kept:
            break
        best = r
        r *= 2
    out["rate_sweep"] = sweep
    out["sustainable_req_per_s"] = best if best is not None else (rate if rps >= 0.95 * rate
                                                                   else None)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the mining path "
              "is single-GPU in this build", file=sys.stderr)
        sys.exit(2)
    # Every input is generated before the GPU library is loaded (the batch in
    # a pool of spawned processes), so no worker is started from a process
    # that holds a GPU context.
    import synth
    t0 = time.time()
    c = synth.config(2)
    others = [] if args.only_headline else [synth.config(1), synth.config(3)]
    batch = ([] if args.only_headline or args.no_batch else
             synth.batch_config(args.batch_count, workers=16))
    small = ([] if args.only_headline or args.no_serve else
             synth.batch_config(16, seed=synth.CONFIG_SEED_BASE + 5, workers=16))
    log(f"inputs generated in {time.time() - t0:.1f}s")
    import paper_1812_10959_amd as dic
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    h = headline(dic, args, c)
    line = {
        "metric": METRIC, "value": round(h["value"], 3), "unit": "G subset-tests/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(h["ms_per_step"], 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "quest_zipf_n1M_m1000", "n": int(h["rows"].shape[0]), "m": c["m"],
                   "minsup": c["minsup"], "M": c["M"], "seed": c["meta"]["seed"],
                   "path": "dic_mine (plain, one database)",
                   "layout": "item_bitsets" if args.layout == 1 else "row_bitmaps"},
        "roofline": h["roofline"],
        "stats": {k: h["stats"][k] for k in ("tau", "stops", "tests", "peak_live", "n_frequent",
                                              "k_max", "known", "restarts")},
        "layouts": h["layouts"],
    }
    if "first_pass" in h:
        line["first_pass"] = h["first_pass"]
    if not args.only_headline:
        line["load_db"] = load_entry(dic, c)
    if not args.only_headline:
        if not args.no_cpu:
            threads = args.cpu_threads if args.cpu_threads else min(16, _host_cpus())
            line["cpu_baseline"] = cpu_baseline(c, h["rows"], args.cpu_rows, max(threads, 0),
                                                h["result"])
        log("other single-database workloads ...")
        line["workloads"] = other_configs(dic, others)
        log("association rules ...")
        line["rules"] = rules_bench(dic, [
            ("quest_zipf_n1M_m1000", h["db"], c),
            ("dense_n500k_m128", dic.dic_load_db(others[1]["rows"], others[1]["m"]), others[1])])
        if not args.no_batch:
            line["batched_vs_plain"] = batch_vs_plain(dic, batch)
        if not args.no_serve:
            line["serving"] = serving(dic, args.serve_seconds, args.serve_rate, c, others[1],
                                      small)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
