#!/usr/bin/env python3
"""Benchmark of the gfx950 word sort: one JSON line on stdout.

A step is one whole sort (length histogram, bucket scatter and packing,
odd-even chunk sort, every merge level) of the workload, with inputs already
in HBM, through the graph-captured plan (the batched form).  Default
workload: 64M words, 1M-word Zipf(1.1) vocabulary, lengths 1-24 (the
largest single-GPU configuration).  Beside it the line carries the
per-bucket-launch form on the same input, the roofline of the dominant
kernel (HIP-event timed on its stream) and the CPU oracle's rate.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4|c3|c2|c1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mwords/s sorted + achieved HBM GB/s, batched vs per-bucket launch, bit-exact"
HBM_PEAK_GBS = 8000.0
PACK_MAX = 1024          # segments of at most this many words are sorted several to a tile
WORKLOADS = {
    "c1": (1, "35k words, 5k-word Zipf(1.0) vocabulary, lengths 1-16"),
    "c2": (2, "250k words, 20k-word Zipf(1.0) vocabulary, lengths 1-20, odd-even chunks of 1024"),
    "c3": (3, "4096 documents of 100-50k words (log-uniform), 50k-word Zipf(1.1) vocabulary, lengths 1-20"),
    "c4": (4, "64M words, 1M-word Zipf(1.1) vocabulary, lengths 1-24"),
    "c5": (5, "serving: Poisson arrivals, request sizes lognormal (median 20k words, 1k-1M), "
              "20k-word Zipf(1.0) vocabulary, lengths 1-20, 8 GiB HBM budget"),
}
CSRC = [os.path.join(ROOT, "paper_1411_5283_amd", "csrc", f)
        for f in ("sw_device.hpp", "sw_keys.hpp", "sw_tiles.hpp", "sw_split.hpp", "sw_window.hpp", "sw_kernels.hpp", "sw_text.hpp",
                  "sw_bytes.hpp", "sw_gather.hpp", "sw_runtime.hip")]
# VALU issue rate of the whole GPU: 256 CUs x 4 SIMDs x 16 lanes per clock
# (a wave64 instruction occupies its SIMD for 4 clocks) x 2.4 GHz, in tera
# lane-operations per second (the fp32 vector figure, 157.3 TFLOP/s, is this
# rate x 2 for fused multiply-add x 2 for dual issue; a sort issues neither).
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def counter_file(kind: str, workload: str) -> str:
    """profiles/hbm_traffic_<workload>.json or profiles/sq_counters_<workload>.json"""
    return os.path.join(ROOT, "profiles", "%s_%s.json" % (kind, workload))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in CSRC:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# ------------------------------------------------------------------ byte model
def element_bytes(cls: int) -> int:
    """HBM bytes of one key element of a class: packed u64, or lanes + u32 index."""
    return {0: 8, 1: 12, 2: 20, 3: 28, 4: 36}[cls]


def class_of_len(L: int) -> int:
    return 0 if L <= 4 else (1 if L <= 8 else (2 if L <= 16 else (3 if L <= 24 else 4)))


def levels_for(n: int, T: int) -> int:
    m, r = 0, T
    while r < n:
        r <<= 1
        m += 1
    return m


def merge_passes(n: int, T: int, fan: int) -> int:
    """HBM merge passes of a segment of n items after tiles of T: two-way
    levels double the run length, four-way passes quadruple it."""
    m = levels_for(n, T)
    return (m + 1) // 2 if fan == 4 else m


def algorithmic_bytes(seg_sizes, tiles, fans=(2, 2, 2, 2, 2)):
    """Bytes each kernel family must move, per step, for the given segments.

    seg_sizes: list of (length L, words n).  tiles[c] = (chunk-sort tile T),
    fans[c] = runs merged per HBM pass (2 or 4).  chunk sort: read the
    element, write it back (or 4-byte index if the segment is finished);
    merge pass p < m: read + write the element, the last pass writes the
    4-byte index instead.  Scatter: 4 B offset + L chars in, one element out.
    Histogram: 4 B offset per word."""
    fam = {}

    def add(k, v):
        fam[k] = fam.get(k, 0) + v

    for L, n in seg_sizes:
        if n == 0:
            continue
        c = class_of_len(L)
        e = element_bytes(c)
        m = levels_for(n, tiles[c])
        add("hist", 4 * n)
        add("scatter_pack", (4 + L + e) * n)
        if n <= PACK_MAX:       # short segments: several to a tile
            add("sort_packed_c%d" % c, (e + 4) * n)
            continue
        add("sort_tiles_c%d" % c, (e + (e if m else 4)) * n)
        passes = merge_passes(n, tiles[c], fans[c])
        for l in range(passes):
            add("merge_c%d" % c, (e + (e if l < passes - 1 else 4)) * n)
    return fam


# ------------------------------------------------------------------ helpers
def light_check(wl, perm: np.ndarray, boff: np.ndarray, n_docs: int) -> dict:
    """Invariants of the result that hold at any size (no oracle): a
    permutation per document, bucket sizes equal the length histogram, and the
    key order on a sample of neighbouring pairs."""
    offs = wl.offsets.astype(np.int64)
    lens = offs[1:] - offs[:-1]
    docs = wl.doc_offsets.astype(np.int64) if wl.doc_offsets is not None else np.array([0, wl.n])
    boff = boff.reshape(n_docs, 34).astype(np.int64)
    rng = np.random.default_rng(0)
    ok = True
    for d in range(n_docs) if n_docs <= 64 else rng.choice(n_docs, 64, replace=False):
        lo, hi = int(docs[d]), int(docs[d + 1])
        p = perm[lo:hi].astype(np.int64)
        ok &= bool(p.size == 0 or (p.max() < hi - lo and np.all(np.bincount(p, minlength=hi - lo) == 1)))
        h = np.bincount(lens[lo:hi], minlength=33)[:33]
        ok &= bool(np.array_equal(np.diff(boff[d]), h) and boff[d][0] == 0)
        if hi - lo > 1:
            k = rng.integers(0, hi - lo - 1, size=min(200_000, hi - lo - 1))
            a, b = p[k] + lo, p[k + 1] + lo
            la, lb = lens[a], lens[b]
            good = la < lb
            same = la == lb
            # compare bytes of equal-length neighbours one by one (sample only)
            for j in range(int(lens.max(initial=0))):
                ca = np.where(la > j, wl.chars[np.minimum(offs[a] + j, len(wl.chars) - 1)], 0)
                cb = np.where(lb > j, wl.chars[np.minimum(offs[b] + j, len(wl.chars) - 1)], 0)
                good |= same & (ca < cb)
                same &= ca == cb
            good |= same & (a < b)
            ok &= bool(np.all(good))
    return {"invariants": "permutation, bucket sizes, key order on sampled neighbours",
            "ok": bool(ok)}


def _grow_sample(wl, fn, budget_s: float, start: int):
    """Time fn(chars, offsets) on ever longer prefixes of the word list until
    one run takes about budget_s / 2.2; a list that is used whole sooner is
    sorted again and again for about budget_s / 4.  Returns (words sorted,
    seconds, runs)."""
    n = min(start, wl.n)
    while True:
        offs = np.ascontiguousarray(wl.offsets[:n + 1])
        t0 = time.perf_counter()
        fn(wl.chars, offs)
        dt = time.perf_counter() - t0
        if dt * 2.2 > budget_s:
            return n, dt, 1
        if n >= wl.n:
            runs = max(1, int(budget_s / 4 / max(dt, 1e-6)))
            t0 = time.perf_counter()
            for _ in range(runs):
                fn(wl.chars, offs)
            return n * runs, time.perf_counter() - t0, runs
        n = min(n * 2, wl.n)


def cpu_baseline(wl, workload: str, budget_s: float = 16.0) -> dict:
    """The oracle as it stands on the host's cores, on bounded prefix samples
    of the same workload: oracle_def (qsort by length, bytes, index) with
    each length list on a thread of its own over every core the process may
    use (the value), the same on one thread, the paper's own method
    (oracle_bubble, one thread) on the stand-in for its first dataset and, for
    the 250k-word workload, on that whole list (Table 1's second dataset), the
    results-table analog, and for a batch of documents both oracles with a
    document a thread."""
    import oracle
    oracle.build(force=False)
    cores = len(os.sched_getaffinity(0))
    n_all, dt_all, r_all = _grow_sample(wl, lambda c, o: oracle.oracle_def_parallel(c, o, threads=cores),
                                        budget_s * 0.6, 1 << 21)
    n_one, dt_one, r_one = _grow_sample(wl, oracle.oracle_def, budget_s * 0.4, 1 << 20)
    what = lambda n, r: ("the whole list (%d words) %d times" % (n // r, r)) if r > 1 else "the first %d words" % n
    legs = {"all_cores": {"value": n_all / dt_all / 1e6, "unit": "Mwords/s", "cores": cores,
                          "sample": "oracle_def_parallel (each length list sorted by oracle_def on its own "
                                    "thread, %d threads) on %s of the same workload, %.2f s" %
                                    (cores, what(n_all, r_all), dt_all)},
            "single_thread": {"value": n_one / dt_one / 1e6, "unit": "Mwords/s", "cores": 1,
                              "sample": "oracle_def on %s of the same workload, %.2f s" %
                                        (what(n_one, r_one), dt_one)}}
    # the faster leg is the baseline (on a small list the threads cost more than they save)
    best = max(legs, key=lambda k: legs[k]["value"])
    res = {"value": legs[best]["value"], "unit": "Mwords/s", "cores": legs[best]["cores"], "kind": "oracle",
           "sample": legs[best]["sample"], "leg": best, **legs}
    from paper_1411_5283_amd import wordgen
    c1 = wordgen.config(1)
    t0 = time.perf_counter()
    oracle.oracle_bubble(c1.chars, c1.offsets)
    res["oracle_bubble_35k_words_s"] = t1 = time.perf_counter() - t0
    res["paper_table1_dataset1_s"] = 6.639
    res["table3_analog_35k_words"] = table3_analog(oracle, c1, t1, [p for p in (2, 4, 6, 8, 10, 16) if p <= cores])
    if wl.doc_offsets is not None:
        res["doc_parallel"] = doc_parallel_baseline(oracle, wl, cores, budget_s)
    if workload == "c2":
        t0 = time.perf_counter()
        oracle.oracle_bubble(wl.chars, wl.offsets)
        res["oracle_bubble_250k_words_s"] = t1 = time.perf_counter() - t0
        res["paper_table1_dataset2_s"] = 188.262
        res["table3_analog_250k_words"] = table3_analog(oracle, wl, t1,
                                                        [p for p in (4, 6, 8, 10, 16) if p <= cores])
    res["paper_hardware"] = "Intel Core i7-3610QM 2.3 GHz (paper, Table 1)"
    try:
        with open("/proc/cpuinfo") as f:
            res["host_cpu"] = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "?")
    except OSError:
        pass
    res["host_cores_available"] = cores
    return res


def _counters(kind: str, kernel: str, workload: str, tiles: dict):
    """The committed rocprofv3 counter summary of one kernel family, if it was
    taken on the current kernel source, on the same workload and with the same
    tile configuration (else None)."""
    try:
        with open(counter_file(kind, workload)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    if t.get("workload", "").split(":")[0].strip() != workload:
        return None
    if t.get("tiles") != tiles:
        return None
    return t.get("kernels", {}).get(kernel)


def doc_parallel_baseline(oracle, wl, cores: int, budget_s: float) -> dict:
    """Documents on host threads (oracle_batch: each document sorted alone, one
    a thread): oracle_def and the paper's method oracle_bubble, each on the
    first documents of the batch that take about budget_s / 4."""
    docs = wl.doc_offsets.astype(np.int64)
    out = {}
    for fn in ("oracle_def", "oracle_bubble"):
        nd = 16
        while True:
            nd = min(nd, wl.n_docs)
            d = docs[:nd + 1]
            offs = np.ascontiguousarray(wl.offsets[:int(d[-1]) + 1])
            t0 = time.perf_counter()
            oracle.oracle_batch(wl.chars, offs, d.astype(np.uint32), fn=fn, threads=cores)
            dt = time.perf_counter() - t0
            if dt * 2.2 > budget_s / 4 or nd >= wl.n_docs:
                break
            nd *= 2
        out[fn] = {"value": int(d[-1]) / dt / 1e6, "unit": "Mwords/s", "cores": cores,
                   "sample": "%s on the first %d documents (%d words), a document a thread, %.2f s" %
                             (fn, nd, int(d[-1]), dt)}
    return out


def table3_analog(oracle, wl, t1: float, ps) -> dict:
    """The paper's parallel method on p host threads, timed like the results
    table of section 5: the words are put into length lists; each list is cut
    into p chunks of ceil(list size / p) words (chunk = array size /
    processors); worker i bubble-sorts chunk i of every list (oracle_bubble
    on the words of its chunks, one thread each), then one thread merges
    every list's chunks.  The merge is timed as oracle_chunked minus
    oracle_chunks at a chunk of ceil(longest list / p) (the same bubble-sorted
    chunks with and without the master's merge).  T_p = the slowest worker +
    the merge; speedup = T_1 / T_p with T_1 = oracle_bubble on the whole list,
    efficiency = 100 * speedup / p (report.py)."""
    from concurrent.futures import ThreadPoolExecutor
    from paper_1411_5283_amd import report
    offs = wl.offsets.astype(np.int64)
    lens = offs[1:] - offs[:-1]
    order = np.argsort(lens, kind="stable")
    counts = np.bincount(lens, minlength=33)
    starts = np.concatenate([[0], np.cumsum(counts)])
    rows = []
    for p in ps:
        parts = []
        for i in range(p):
            idx = []
            for L in range(33):
                n_l = int(counts[L])
                if n_l == 0:
                    continue
                c = oracle.paper_chunk_size(n_l, p)
                idx.append(order[starts[L] + min(i * c, n_l):starts[L] + min((i + 1) * c, n_l)])
            idx = np.concatenate(idx) if idx else np.zeros(0, np.int64)
            sub_l = lens[idx]
            sub_o = np.concatenate([[0], np.cumsum(sub_l)]).astype(np.uint32)
            pos = (offs[idx][:, None] + np.arange(33)[None, :])
            keep = np.arange(33)[None, :] < sub_l[:, None]
            sub_c = wl.chars[np.minimum(pos[keep], max(len(wl.chars) - 1, 0))] if keep.any() else \
                np.zeros(1, np.uint8)
            parts.append((np.ascontiguousarray(sub_c), sub_o))
        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=p) as ex:
            list(ex.map(lambda a: oracle.oracle_bubble(*a), parts))
        t_chunks = time.perf_counter() - t0
        c = oracle.paper_chunk_size(int(counts.max()), p)
        t0 = time.perf_counter()
        oracle.oracle_chunked(wl.chars, wl.offsets, c)
        t_whole = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.oracle_chunks(wl.chars, wl.offsets, c)
        t_merge = max(t_whole - (time.perf_counter() - t0), 0.0)
        tp = t_chunks + t_merge
        rows.append({"p": p, "chunk_step_s": t_chunks, "merge_s": t_merge, "T_p_s": tp,
                     "speedup": report.speedup(t1, tp), "efficiency_pct": report.efficiency(t1, tp, p)})
    return {"T_1_s": t1, "rows": rows,
            "method": "chunk step on p threads (chunk i of every length list on thread i, chunk = "
                      "ceil(list size / p)), then the merge on one thread; T_1 = oracle_bubble"}


def hbm_traffic(kernel: str, workload: str, tiles: dict):
    """HBM bytes per launch of a kernel family (FETCH_SIZE + WRITE_SIZE, scaled
    by a plain copy's reading), or None."""
    k = _counters("hbm_traffic", kernel, workload, tiles)
    return None if k is None else k.get("bytes_per_launch")


def alu_roofline(kernel: str, info: dict, workload: str, tiles: dict, fam_bytes: dict) -> dict:
    """VALU view of a chunk-sort kernel: issued VALU lane-operations per launch
    (SQ_INSTS_VALU x 64, from the committed counter summary of the same source,
    workload and tiles) over the launch time measured live with HIP events."""
    sq = _counters("sq_counters", kernel, workload, tiles)
    us = info["avg_launch_us"]
    launches = info["launches_per_step"]
    r = {"bound": "alu", "kernel": kernel, "achieved": None, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
         "frac": None, "traffic": hbm_traffic(kernel, workload, tiles), "avg_launch_us": us,
         "algorithmic_bytes_per_launch": (fam_bytes.get(kernel, 0) / launches) if launches else None,
         "what": "VALU lane-operations issued per second (wave instructions x 64 lanes); peak = 256 CUs x "
                 "64 lanes x 2.4 GHz"}
    if r["algorithmic_bytes_per_launch"]:
        r["hbm_frac"] = r["algorithmic_bytes_per_launch"] / (us * 1e-6) / 1e9 / HBM_PEAK_GBS
    if sq is None:
        r["counters"] = None
        return r
    valu = sq.get("SQ_INSTS_VALU_per_dispatch")
    if valu:
        r["achieved"] = valu * 64 / (us * 1e-6) / 1e12
        r["frac"] = r["achieved"] / VALU_PEAK_TOPS
    # GRBM_GUI_ACTIVE is summed over the 8 XCDs: / 8 = the dispatch's clocks
    cyc = sq["GRBM_GUI_ACTIVE_per_dispatch"] / 8 if sq.get("GRBM_GUI_ACTIVE_per_dispatch") else None
    names = ("SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_THREAD_CYCLES_VALU", "SQ_ACTIVE_INST_VALU2", "SQ_INSTS_LDS",
             "SQ_ACTIVE_INST_LDS", "SQ_LDS_IDX_ACTIVE", "SQ_LDS_BANK_CONFLICT", "SQ_WAIT_INST_LDS", "SQ_WAVES",
             "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_INSTS_SALU", "GRBM_GUI_ACTIVE")
    r["counters"] = {k: sq.get(k + "_per_dispatch") for k in names}
    if cyc:
        r["clock_GHz"] = cyc / (us * 1e-6) / 1e9
        # quad-cycles summed over waves, over the 1024 SIMDs for the dispatch's clocks
        if sq.get("SQ_ACTIVE_INST_VALU_per_dispatch"):
            r["valu_busy"] = sq["SQ_ACTIVE_INST_VALU_per_dispatch"] * 4 / (1024 * cyc)
        if sq.get("SQ_ACTIVE_INST_LDS_per_dispatch"):
            r["lds_busy"] = sq["SQ_ACTIVE_INST_LDS_per_dispatch"] * 4 / (1024 * cyc)
    if sq.get("SQ_THREAD_CYCLES_VALU_per_dispatch") and sq.get("SQ_ACTIVE_INST_VALU_per_dispatch"):
        r["valu_lane_util"] = sq["SQ_THREAD_CYCLES_VALU_per_dispatch"] / \
            (sq["SQ_ACTIVE_INST_VALU_per_dispatch"] * 64)
    if sq.get("SQ_INSTS_LDS_per_dispatch"):
        r["lds_conflict_cycles_per_lds_inst"] = sq.get("SQ_LDS_BANK_CONFLICT_per_dispatch", 0) / \
            sq["SQ_INSTS_LDS_per_dispatch"]
    return r


# ------------------------------------------------------------------ serving
def serve_bench(args, sw, wordgen, torch):
    """Continuous batching under Poisson arrivals: the library's native serving
    loop (sw_server_*), or with --serve-python the Python scheduler of
    paper_1411_5283_amd/serve.py."""
    n_warm, n_meas = args.serve_warmup, args.serve_requests
    log("generating %d requests" % (n_warm + n_meas))
    reqs = list(wordgen.serving_requests(n_warm + n_meas))
    warm, meas = reqs[:n_warm], reqs[n_warm:]
    if args.serve_python:
        out, ex = serve_python(args, sw, reqs, warm, meas)
        loop = "python scheduler (serve.py) over graph-captured plans"
    else:
        out, ex = serve_native(args, sw, reqs, warm, meas)
        loop = "native serving loop (sw_server_*: C++ scheduler thread, pinned staging, %d copy threads)" % \
            args.serve_copy_threads
    sat, points, budget = out
    main_pt = points[1]
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        from concurrent.futures import ThreadPoolExecutor
        cores = len(os.sched_getaffinity(0))
        t0 = time.perf_counter()
        nw = 0
        # requests in arrival order, each sorted by oracle_def on a thread of its own
        with ThreadPoolExecutor(max_workers=cores) as ex:
            for k0 in range(0, len(meas), cores):
                part = meas[k0:k0 + cores]
                list(ex.map(lambda r: oracle.oracle_def(r.chars, r.offsets), part))
                nw += sum(r.n for r in part)
                if time.perf_counter() - t0 > 10:
                    break
        dt = time.perf_counter() - t0
        cpu = {"value": nw / dt / 1e6, "unit": "Mwords/s", "cores": cores, "kind": "oracle",
               "sample": "oracle_def on the measured requests in arrival order, one request a thread on %d "
                         "threads, until 10 s (%d words)" % (cores, nw)}
    sizes = np.array([r.n for r in meas])
    return {
        "metric": METRIC, "value": main_pt["mwords_s"], "unit": "Mwords/s", "n_gpus": 1,
        "steps": len(meas), "warmup": len(warm), "ms_per_step": main_pt["seconds"] * 1e3 / len(meas),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "c5: " + WORKLOADS["c5"][1], "request_median": float(np.median(sizes)),
                   "request_mean": float(sizes.mean()), "slots": args.serve_slots,
                   "max_batch_words": args.serve_batch_words, "budget_bytes": budget,
                   "min_batch_words": args.serve_min_words, "max_wait_ms": args.serve_max_wait_ms,
                   "loop": loop, "value_at": "lambda = 0.8 x closed-burst saturation rate",
                   "passes": "each point: median by throughput of %d passes of the %d measured requests" %
                             (args.serve_passes, len(meas))},
        "serving": {"saturation": sat, "points": points},
        "roofline": None, "cpu_baseline": cpu, "kernel_source": kernel_source_hash(),
    }


def _arrivals(rset, rate, submit):
    """Submit every request at Poisson times (rate None: all at once); returns the start time."""
    rng = np.random.default_rng(1)
    t0 = time.perf_counter()
    if rate is None:
        return t0, [submit(r) for r in rset]
    t = t0
    out = []
    for r in rset:
        t += rng.exponential(1.0 / rate)
        wait = t - time.perf_counter()
        if wait > 3e-4:                 # sleep most of a long gap, spin the rest (sleep is coarse)
            time.sleep(wait - 2e-4)
        while time.perf_counter() < t:
            pass
        out.append(submit(r))
    return t0, out


def _serve_points(run, warm, meas):
    sat = run(warm, None)
    log("saturation (closed burst): %s" % sat)
    sat_rate = sat["requests"] / sat["seconds"]
    points = []
    for frac in (0.5, 0.8, 1.0):
        r = run(meas, frac * sat_rate)
        r["lambda_req_s"] = frac * sat_rate
        r["lambda_frac"] = frac
        points.append(r)
        log("lambda %.1f x saturation: %s" % (frac, r))
    return sat, points


def serve_native(args, sw, reqs, warm, meas):
    """One server for the whole measurement: the warm-up requests go first
    (a closed burst, not measured), then the saturation rate is a closed burst
    of the measured requests, then Poisson arrivals at fractions of it."""
    cfg = dict(slots=args.serve_slots, max_batch_words=args.serve_batch_words,
               max_batch_docs=args.serve_batch_docs, max_batch_chars=args.serve_batch_words * 8,
               min_batch_words=args.serve_min_words, max_wait_us=int(args.serve_max_wait_ms * 1e3),
               copy_threads=args.serve_copy_threads)
    probe = sw.NativeServer(budget_bytes=1 << 30, **cfg)
    budget = (8 << 30) - probe.fixed_bytes()
    probe.close()
    srv = sw.NativeServer(budget_bytes=budget, **cfg)

    def run(rset, rate):
        s0 = srv.stats()
        t0, tickets = _arrivals(rset, rate, lambda r: srv.submit(r.chars, r.offsets))
        lats = [srv.wait(t)[2] for t in tickets]
        t1 = time.perf_counter()
        s1 = srv.stats()
        words = sum(r.n for r in rset)
        return {"requests": len(rset), "words": words, "seconds": t1 - t0,
                "mwords_s": words / (t1 - t0) / 1e6, "p50_ms": float(np.percentile(lats, 50)) * 1e3,
                "p99_ms": float(np.percentile(lats, 99)) * 1e3, "batches": s1["batches"] - s0["batches"],
                "max_bytes_in_use": s1["max_bytes_in_use"]}

    def median_of(k, rset, rate):
        # one pass of the measured requests takes tens of milliseconds: the
        # median (by throughput) of k passes, with every pass kept
        rs = sorted((run(rset, rate) for _ in range(k)), key=lambda r: r["mwords_s"])
        out = dict(rs[k // 2])
        out["passes"] = [{q: r[q] for q in ("mwords_s", "p50_ms", "p99_ms", "batches")} for r in rs]
        return out

    run(warm, None)
    sat = median_of(args.serve_passes, meas, None)
    log("saturation (closed burst of the measured requests): %s" % sat)
    sat_rate = sat["requests"] / sat["seconds"]
    points = []
    for frac in (0.5, 0.8, 1.0):
        r = median_of(args.serve_passes, meas, frac * sat_rate)
        r["lambda_req_s"] = frac * sat_rate
        r["lambda_frac"] = frac
        points.append(r)
        log("lambda %.1f x saturation: %s" % (frac, r))
    st = srv.stats()
    srv.close()
    assert st["max_bytes_in_use"] <= budget
    return (sat, points, budget), None


def serve_python(args, sw, reqs, warm, meas):
    from paper_1411_5283_amd.serve import GpuExecutor, SortServer
    ex = GpuExecutor(slots=args.serve_slots, max_batch_words=args.serve_batch_words,
                     max_batch_docs=args.serve_batch_docs, max_batch_chars=args.serve_batch_words * 8)
    budget = (8 << 30) - ex.fixed_bytes()

    def run(rset, rate):
        srv = SortServer(ex, budget_bytes=budget, max_batch_words=args.serve_batch_words,
                         max_batch_docs=args.serve_batch_docs, min_batch_words=args.serve_min_words,
                         max_wait_s=args.serve_max_wait_ms * 1e-3)
        srv.start()
        t0, futs = _arrivals(rset, rate, lambda r: srv.submit(r.chars, r.offsets))
        for f in futs:
            f.result(timeout=300)
        t1 = time.perf_counter()
        srv.stop()
        words = sum(r.n for r in rset)
        return {"requests": len(rset), "words": words, "seconds": t1 - t0,
                "mwords_s": words / (t1 - t0) / 1e6, "p50_ms": srv.stats.percentile(50) * 1e3,
                "p99_ms": srv.stats.percentile(99) * 1e3, "batches": srv.stats.batches,
                "max_bytes_in_use": srv.stats.max_bytes_in_use}

    out = (*_serve_points(run, warm, meas), budget)
    ex.close()
    return out, None


def text_bench(args, sw, wordgen, torch, wl, chars, offs, docs, perm, boff, perm_h, boff_h, stream, plan,
               plan_ms, tile_cfg):
    """The steps around the sort on the same workload: the word list written as
    raw text (capitals, punctuation, line breaks) is tokenized back on the GPU
    (lower-case folding), and the sorted result is written out as text with a
    line break after every word, from the permutation (sort_words_materialize)
    and in the sort's own pass from the sorted keys (sw_plan_run_text).  All
    are timed with HIP events on the bench stream and checked (the tokenized
    list must equal the word list; sampled words of the sorted text must equal
    the words perm names; the one-pass text must equal the other byte for
    byte, and its permutation the plan's)."""
    n, nd = wl.n, wl.n_docs
    dev = chars.device
    t0 = time.perf_counter()
    raw = wordgen.render_text(wl, 14115283)
    log("rendered %d bytes of text in %.1f s" % (raw.size, time.perf_counter() - t0))
    reps = 5
    text = torch.from_numpy(raw).to(dev)
    nb = raw.size
    tchars = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
    toffs = torch.empty(n + 2, dtype=torch.int32, device=dev)
    tnw = torch.zeros(1, dtype=torch.int32, device=dev)
    tws = torch.empty(sw.tokenize_workspace_size(nb), dtype=torch.uint8, device=dev)
    run_tok = lambda: sw.tokenize(text, nb, sw.TOK_LOWER, tchars, toffs, n + 1, tnw, tws, stream)
    run_tok()
    sw.sort_words_status(tws, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        run_tok()
    e1.record(stream)
    torch.cuda.synchronize()
    sw.sort_words_status(tws, stream)
    tok_ms = e0.elapsed_time(e1) / reps
    nw = int(tnw.cpu()[0])
    letters = int(offs[n].item()) - int(offs[0].item()) if n else 0
    tok_ok = nw == n and bool(torch.equal(toffs[:n + 1], offs[:n + 1] - offs[0])) and \
        bool(torch.equal(tchars[:letters], chars[:letters]))
    tok_bytes = 2 * nb + letters + 4 * (nw + 1)      # text read twice, letters and offsets written
    log("tokenize: %.3f ms, %d words, same=%s" % (tok_ms, nw, tok_ok))
    del text, tchars, toffs, tws

    size = letters + n
    out = torch.empty(max(size, 1), dtype=torch.uint8, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    run_mat = lambda: sw.materialize(chars, offs, docs, nd, n, perm, boff, 10, out, st, stream)
    run_mat()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        run_mat()
    e1.record(stream)
    torch.cuda.synchronize()
    mat_ms = e0.elapsed_time(e1) / reps
    status = int(st.cpu()[0])
    # sampled check: the text of a few hundred sorted positions
    rng = np.random.default_rng(5)
    ks = rng.integers(0, n, 300) if n else []
    out_h = out.cpu().numpy()
    doc_h = wl.doc_offsets if wl.doc_offsets is not None else np.array([0, n], np.uint32)
    bo = boff_h[:nd * 34].reshape(nd, 34).astype(np.int64)
    mat_ok = status == 0
    for k in ks:
        d = int(np.searchsorted(doc_h, k, side="right") - 1)
        kl = int(k) - int(doc_h[d])
        L = int(np.searchsorted(bo[d], kl, side="right") - 1)
        cnt = np.diff(bo[d])
        pos = int(wl.offsets[doc_h[d]]) - int(wl.offsets[0]) + int(doc_h[d])
        pos += int(sum(int(cnt[l]) * (l + 1) for l in range(L))) + (kl - int(bo[d][L])) * (L + 1)
        i = int(doc_h[d]) + int(perm_h[k])
        w = wl.chars[wl.offsets[i]:wl.offsets[i + 1]].tobytes()
        mat_ok &= out_h[pos:pos + L + 1].tobytes() == w + b"\n"
    mat_bytes = 4 * n + 8 * n + letters + size       # perm, offsets, characters, text
    log("materialize: %.3f ms, status=%d, sampled check=%s" % (mat_ms, status, mat_ok))

    # sort and text in one pass: the sorted keys are written out as text
    out2 = torch.empty(max(size, 1), dtype=torch.uint8, device=dev)
    perm4 = torch.empty_like(perm)
    run_st = lambda: plan.run_text(chars, offs, docs, nd, n, perm4, boff, 10, out2)
    run_st()
    st_status = plan.status_code()
    e0.record(stream)
    for _ in range(reps):
        run_st()
    e1.record(stream)
    torch.cuda.synchronize()
    st_ms = e0.elapsed_time(e1) / reps
    st_status = st_status or plan.status_code()
    st_same = st_status == 0 and bool(torch.equal(out2[:size], out[:size])) and bool(torch.equal(perm4, perm))
    log("sort + text: %.3f ms (sort alone %.3f ms), status=%d, same text and permutation=%s" %
        (st_ms, plan_ms, st_status, st_same))
    del out, out2, perm4
    return {
        "tokenize": {"ms": tok_ms, "text_bytes": nb, "words": nw, "Mwords_per_s": nw / (tok_ms / 1e3) / 1e6,
                     "algorithmic_GBs": tok_bytes / (tok_ms / 1e3) / 1e9, "same_as_word_list": tok_ok,
                     "traffic_bytes": {k: hbm_traffic(k, args.workload, tile_cfg) for k in ("tok_sum", "tok_scan", "tok_write")},
                     "input": "the word list rendered as text: capitals, punctuation, line breaks, digits"},
        "materialize": {"ms": mat_ms, "text_bytes": size, "Mwords_per_s": n / (mat_ms / 1e3) / 1e6,
                        "algorithmic_GBs": mat_bytes / (mat_ms / 1e3) / 1e9, "status": status,
                        "traffic_bytes": hbm_traffic("materialize", args.workload, tile_cfg),
                        "sampled_check": bool(mat_ok), "separator": "line feed"},
        "sort_and_text": {"ms": st_ms, "sort_alone_ms": plan_ms, "text_ms": st_ms - plan_ms,
                          "Mwords_per_s": n / (st_ms / 1e3) / 1e6, "status": st_status,
                          "same_text_as_materialize": st_same,
                          "traffic_bytes": hbm_traffic("keys_text", args.workload, tile_cfg),
                          "form": "sw_plan_run_text: the sort's graph plus the text written from the sorted "
                                  "keys (each segment's last level also keeps its keys)"},
    }


# ------------------------------------------------------------------ counter calibration
def copy_calibration(torch, nbytes: int = 1 << 30):
    """A plain device copy of a known size, three times (read nbytes, write nbytes)."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 3}), flush=True)


# ------------------------------------------------------------------ main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--clock-ramp-s", type=float, default=0.25,
                    help="untimed replays for this many seconds before the warmup steps (clock ramp)")
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--profile-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--untuned", action="store_true", help="ignore the autotuner cache")
    ap.add_argument("--no-text", action="store_true",
                    help="skip the tokenizer and sorted-text measurements around the sort")
    ap.add_argument("--serial", action="store_true",
                    help="run the key classes one after another (for per-kernel profiling)")
    ap.add_argument("--merge", default=None,
                    help="merge choice per class, e.g. 0,0,0,0 (two-way levels) or 1,1,1,1 (four-way); "
                         "default: the tuned or built-in choice")
    ap.add_argument("--chunk", default=None,
                    help="chunk size per class, e.g. 16,16,16,32,32; default: the tuned or built-in choice")
    ap.add_argument("--variant", default=None,
                    help="tile configuration per class, e.g. 3,3,1,0,0; default: the tuned or built-in choice")
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-passes", type=int, default=3,
                    help="passes of the measured requests per arrival rate (the median is reported)")
    ap.add_argument("--serve-slots", type=int, default=2)
    ap.add_argument("--serve-batch-words", type=int, default=1 << 22)
    ap.add_argument("--serve-batch-docs", type=int, default=128)
    ap.add_argument("--serve-min-words", type=int, default=1 << 18)
    ap.add_argument("--serve-max-wait-ms", type=float, default=1.0)
    ap.add_argument("--serve-copy-threads", type=int, default=10)
    ap.add_argument("--serve-python", action="store_true", help="the Python scheduler instead of the native loop")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB on the device three times: run under rocprofv3 --pmc FETCH_SIZE "
                         "(then WRITE_SIZE), what the counters read for a copy of known size scales the "
                         "sort's counters into HBM bytes")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU; --gpus %d is not supported (sharding across "
              "GPUs is a design, not code)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.profile_steps < 1 or args.warmup < 0:
        ap.error("--steps and --profile-steps must be at least 1, --warmup at least 0")

    import torch
    if args.copy_calibration:
        copy_calibration(torch)
        return
    import paper_1411_5283_amd as sw
    from paper_1411_5283_amd import wordgen

    if args.workload == "c5":
        torch.cuda.set_device(0)
        print(json.dumps(serve_bench(args, sw, wordgen, torch)), flush=True)
        return
    cfg_no, desc = WORKLOADS[args.workload]
    log("generating workload %s: %s" % (args.workload, desc))
    t0 = time.perf_counter()
    wl = wordgen.config(cfg_no)
    log("generated %d words in %.1f s" % (wl.n, time.perf_counter() - t0))
    tuned = None
    if not args.untuned:
        from paper_1411_5283_amd import tune
        tuned = tune.apply(args.workload)
    if "chunk" in wl.meta:
        # the workload fixes the chunk size (section 5's chunk of the 250k-word
        # list); tiles and launch order as tuned with that chunk, if they were
        sw.set_config(chunk=[wl.meta["chunk"]] * sw.NUM_CLASSES,
                      **({} if tuned else {"variant": [0] * sw.NUM_CLASSES}))
    if args.serial:
        sw.set_config(flags=sw.get_config()["flags"] | sw.FLAG_SERIAL_CLASSES)
    if args.merge:
        sw.set_config(merge=[int(x) for x in args.merge.split(",")])
    if args.variant:
        sw.set_config(variant=[int(x) for x in args.variant.split(",")])
    if args.chunk:
        sw.set_config(chunk=[int(x) for x in args.chunk.split(",")])
    cfg = sw.get_config()
    tiles = [sw.variant_tiles(c, cfg["variant"][c])[0] for c in range(sw.NUM_CLASSES)]
    tile_cfg = {"chunk": list(cfg["chunk"]), "variant": list(cfg["variant"]), "merge": list(cfg["merge"])}

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    chars, offs, docs = sw.device_words(wl, dev)
    n, nd = wl.n, wl.n_docs
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    boff = torch.empty(nd * 34, dtype=torch.int32, device=dev)
    # one dedicated stream: the plan's graph, the eager launches and the timing events share it
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    torch.cuda.synchronize()

    # ---- batched form: graph-captured plan
    plan = sw.Plan(n, nd, stream=stream)
    run = lambda: plan.run(chars, offs, docs, nd, n, perm, boff)
    # a GPU that has been idle runs a short pass at a lower clock: untimed
    # replays for a fixed stretch of wall time bring it to its working clock
    # before the warmup steps (a sub-millisecond pass otherwise times at the
    # idle clock)
    ramp_runs, t_ramp = 0, time.perf_counter()
    while time.perf_counter() - t_ramp < args.clock_ramp_s:
        for _ in range(8):
            run()
        ramp_runs += 8
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        run()
    plan.status()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        run()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.status()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    value = n / (ms_step / 1e3) / 1e6
    log("plan: %.3f ms/step, %.1f Mwords/s (wall %.3f ms/step)" % (ms_step, value, wall * 1e3 / args.steps))

    perm_h = sw.to_u32(perm)[:n]
    boff_h = sw.to_u32(boff)
    check = None if args.no_check else light_check(wl, perm_h, boff_h, nd)
    if check:
        log("check: %s" % check)

    # ---- per-bucket-launch form on the same input
    plain = None
    ws = torch.empty(sw.sort_words_workspace_size(n, nd), dtype=torch.uint8, device=dev)
    doc_t = docs if docs is not None else torch.tensor(np.array([0, n], np.uint32).view(np.int32), device=dev)
    if not args.no_plain and args.plain_steps > 0:
        perm2 = torch.empty_like(perm)
        sw.sort_words_plain(chars, offs, doc_t, nd, perm2, boff, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            sw.sort_words_plain(chars, offs, doc_t, nd, perm2, boff, ws)
        torch.cuda.synchronize()
        pms = (time.perf_counter() - t0) * 1e3 / args.plain_steps
        same = bool(torch.equal(perm2, perm))
        plain = {"value": n / (pms / 1e3) / 1e6, "unit": "Mwords/s", "ms_per_step": pms,
                 "same_result_as_batched": same,
                 "form": "sort_words_plain: histogram read back, chunk sort and each merge level "
                         "launched per (document, length) segment"}
        log("plain: %.3f ms/step, %.1f Mwords/s, same=%s" % (pms, plain["value"], same))
        del perm2

    # ---- baseline without length lists (one key per word, length first; single document)
    unb = None
    if docs is None and not args.no_plain:
        perm3 = torch.empty_like(perm)
        boff3 = torch.empty(34, dtype=torch.int32, device=dev)
        try:
            sw.sort_words_unbucketed(chars, offs, n, perm3, boff3, ws, stream)
            sw.sort_words_status(ws, stream)
            ev0.record(stream)
            for _ in range(args.plain_steps):
                sw.sort_words_unbucketed(chars, offs, n, perm3, boff3, ws, stream)
            ev1.record(stream)
            torch.cuda.synchronize()
            sw.sort_words_status(ws, stream)
            ums = ev0.elapsed_time(ev1) / args.plain_steps
            same = bool(torch.equal(perm3, perm))
            unb = {"value": n / (ums / 1e3) / 1e6, "unit": "Mwords/s", "ms_per_step": ums,
                   "same_result_as_batched": same,
                   "form": "sort_words_unbucketed: one 32-byte key per word (length first), the whole "
                           "list chunk-sorted and merged as one sequence"}
            log("unbucketed: %.3f ms/step, %.1f Mwords/s, same=%s" % (ums, unb["value"], same))
        except sw.SortWordsError as e:
            unb = {"error": str(e)}
        del perm3, boff3

    # ---- the same pass launched eagerly (no graph), classes forked onto side streams
    def eager():
        if docs is None:
            sw.sort_words_ex(chars, offs, n, perm, boff, ws, stream)
        else:
            sw.sort_words_batch(chars, offs, docs, nd, perm, boff, ws, stream)
    eager()
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.profile_steps):
        eager()
    ev1.record(stream)
    torch.cuda.synchronize()
    eager_ms = ev0.elapsed_time(ev1) / args.profile_steps
    log("eager: %.3f ms/step" % eager_ms)

    # ---- per-kernel timing of the same pass (eager launches, HIP events on this stream)
    sw.profile_reset()
    sw.profile_enable(True)
    for _ in range(args.profile_steps):
        if docs is None:
            sw.sort_words_ex(chars, offs, n, perm, boff, ws, stream)
        else:
            sw.sort_words_batch(chars, offs, docs, nd, perm, boff, ws, stream)
    torch.cuda.synchronize()
    prof = sw.profile_read()
    sw.profile_enable(False)
    sw.sort_words_status(ws, stream)

    # algorithmic bytes from the (document, length) segment sizes of the result
    bo = boff_h[:nd * 34].reshape(nd, 34).astype(np.int64)
    segs = [(L, int(c)) for row in np.diff(bo, axis=1) for L, c in enumerate(row)]
    fam_bytes = algorithmic_bytes(segs, tiles, [4 if m else 2 for m in cfg["merge"]])
    kern = {}
    for name, (launches, ms) in prof.items():
        if launches == 0:
            continue
        per_step_ms = ms / args.profile_steps
        b = fam_bytes.get(name)
        kern[name] = {"launches_per_step": launches // args.profile_steps, "ms_per_step": per_step_ms,
                      "avg_launch_us": ms / launches * 1e3}
        if b is not None and per_step_ms > 0:
            kern[name]["algorithmic_GBs"] = b / (per_step_ms / 1e3) / 1e9
    dom = max(kern, key=lambda k: kern[k]["ms_per_step"])
    dom_launches = kern[dom]["launches_per_step"]
    achieved = kern[dom].get("algorithmic_GBs")
    tsum = sum(v["ms_per_step"] for v in kern.values())
    total_bytes = sum(fam_bytes.values())
    traffic = hbm_traffic(dom, args.workload, tile_cfg)
    chunk_fams = [k for k in kern if k.startswith("sort_tiles") or k.startswith("sort_packed")]
    if dom in chunk_fams:
        roof = alu_roofline(dom, kern[dom], args.workload, tile_cfg, fam_bytes)
    else:
        roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                "traffic": traffic,
                "algorithmic_bytes_per_launch": (fam_bytes.get(dom, 0) / dom_launches) if dom_launches else None,
                "avg_launch_us": kern[dom]["avg_launch_us"]}
    # the chunk sort (the paper's bubble-sort step) in its own bound, whichever kernel dominates
    chunk_top = max(chunk_fams, key=lambda k: kern[k]["ms_per_step"]) if chunk_fams else None
    roof.update({
        "kernels": kern,
        "chunk_sort": alu_roofline(chunk_top, kern[chunk_top], args.workload, tile_cfg, fam_bytes)
        if chunk_top else None,
        "whole_pass_algorithmic_GB": total_bytes / 1e9,
        "whole_pass_GBs_at_plan_time": total_bytes / (ms_step / 1e3) / 1e9,
        "whole_pass_frac": total_bytes / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS,
        "eager_kernel_sum_ms": tsum})
    # the compulsory floor of any method (read the offsets and the characters,
    # write the permutation) and the counters' bytes over the whole pass
    floor = 8 * n + int(wl.offsets[-1]) - int(wl.offsets[0])
    roof["floor_GB"] = floor / 1e9
    roof["floor_frac_at_plan_time"] = floor / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS
    per_launch = {k: hbm_traffic(k, args.workload, tile_cfg) for k in kern}
    if kern and all(v is not None for k, v in per_launch.items() if kern[k]["ms_per_step"] > 0.02):
        counted = sum(v * kern[k]["launches_per_step"] for k, v in per_launch.items() if v is not None)
        roof["whole_pass_counter_GB"] = counted / 1e9
        roof["whole_pass_counter_GBs_at_plan_time"] = counted / (ms_step / 1e3) / 1e9

    text = None if args.no_text else text_bench(args, sw, wordgen, torch, wl, chars, offs, docs, perm, boff,
                                                   perm_h, boff_h, stream, plan, ms_step, tile_cfg)
    cpu = None if args.no_cpu_baseline else cpu_baseline(wl, args.workload)
    out = {
        "metric": METRIC, "value": value, "unit": "Mwords/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "clock_ramp": {"seconds": args.clock_ramp_s, "untimed_runs": ramp_runs},
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "%s: %s" % (args.workload, desc), "n_words": n, "n_docs": nd,
                   "form": "graph-captured plan (batched, device-side segment scheduling)",
                   "chunk": cfg["chunk"], "variant": cfg["variant"], "merge": cfg["merge"], "sort_tile": tiles,
                   "tuned": tuned is not None, "classes": "serial" if args.serial else "parallel streams",
                   "short_segments": "before the chunk sort" if cfg["flags"] & sw.FLAG_PACKED_FIRST
                   else "after the chunk sort",
                   "segment_scheduling": "beside the scatter" if cfg["flags"] & sw.FLAG_SCHEDULE_BESIDE_SCATTER
                   else "before the scatter",
                   "class_order": sw.class_order((cfg["flags"] & sw.FLAG_ORDER_MASK) >> sw.FLAG_ORDER_SHIFT)},
        "eager_ms_per_step": eager_ms,
        "per_bucket_launch": plain,
        "batched_over_plain": (value / plain["value"]) if plain else None,
        "unbucketed": unb,
        "batched_over_unbucketed": (value / unb["value"]) if unb and "value" in unb else None,
        "check": check,
        "roofline": roof,
        "around_the_sort": text,
        "cpu_baseline": cpu,
        "kernel_source": kernel_source_hash(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
