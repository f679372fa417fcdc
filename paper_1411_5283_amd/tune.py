"""Autotuner for the chunk size and tile variant of each key class.

For every key class it times each compiled tile variant with each chunk size
on a real workload (kernel time of that class's chunk sort and
merge levels, from the library's HIP-event timing), checks that every
candidate returns exactly the same permutation and bucket offsets as the
first run, and keeps the fastest.  A second stage then times the whole
graph-captured plan, where the classes run side by side (a VALU-bound chunk
sort of one class overlaps the HBM-bound merges of another, which kernel
times taken one at a time cannot see): class by class, each variant is
timed in interleaved rounds and the one with the lowest median plan time is
kept if it beats the current one by more than 0.5 %.  Results are cached in
a JSON file keyed by GPU architecture, compute-unit count and library
version, one entry per workload name.

    python -m paper_1411_5283_amd.tune --workload c4 [--plan-only]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import NUM_CLASSES

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.environ.get("SW_TUNE_CACHE", os.path.join(HERE, "tuned.json"))
CHUNKS = (8, 16, 32, 64, 128, 256)


def device_key() -> str:
    import torch
    import paper_1411_5283_amd as sw
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(p, "gcnArchName", "unknown").split(":")[0]
    return "%s/%dcu/%s" % (arch, p.multi_processor_count, sw.version())


def _run_once(sw, chars, offs, docs, n, nd, perm, boff, ws, stream):
    if docs is None:
        sw.sort_words_ex(chars, offs, n, perm, boff, ws, stream)
    else:
        sw.sort_words_batch(chars, offs, docs, nd, perm, boff, ws, stream)


def tune(wl, name: str, reps: int = 2, chunks=CHUNKS, log=print) -> dict:
    import torch
    import paper_1411_5283_amd as sw

    dev = torch.device("cuda", torch.cuda.current_device())
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    chars, offs, docs = sw.device_words(wl, dev)
    n, nd = wl.n, wl.n_docs
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    boff = torch.empty(nd * 34, dtype=torch.int32, device=dev)
    ws = torch.empty(sw.sort_words_workspace_size(n, nd), dtype=torch.uint8, device=dev)
    start = sw.get_config()
    best = {"chunk": list(start["chunk"]), "variant": list(start["variant"])}

    _run_once(sw, chars, offs, docs, n, nd, perm, boff, ws, stream)
    sw.sort_words_status(ws, stream)
    ref_perm, ref_boff = perm.clone(), boff.clone()
    trials = []
    for c in range(NUM_CLASSES):
        best_t = None
        for v in range(sw.num_variants(c)):
            for C in chunks:
                cfg = {"chunk": list(best["chunk"]), "variant": list(best["variant"])}
                cfg["chunk"][c], cfg["variant"][c] = C, v
                sw.set_config(**cfg)
                _run_once(sw, chars, offs, docs, n, nd, perm, boff, ws, stream)   # warm
                sw.profile_reset()
                sw.profile_enable(True)
                for _ in range(reps):
                    _run_once(sw, chars, offs, docs, n, nd, perm, boff, ws, stream)
                torch.cuda.synchronize()
                prof = sw.profile_read()
                sw.profile_enable(False)
                sw.sort_words_status(ws, stream)
                same = bool(torch.equal(perm, ref_perm) and torch.equal(boff, ref_boff))
                if not same:
                    raise RuntimeError("class %d variant %d chunk %d changed the result" % (c, v, C))
                ms = sum(prof.get(k, (0, 0.0))[1] for k in
                         ("sort_tiles_c%d" % c, "merge_c%d" % c)) / reps
                trials.append({"class": c, "variant": v, "chunk": C, "ms": ms})
                log("class %d variant %d chunk %4d: %.4f ms" % (c, v, C, ms))
                if best_t is None or ms < best_t:
                    best_t = ms
                    bc, bv = C, v
        best["chunk"][c], best["variant"][c] = bc, bv
        sw.set_config(**best)
    total = 0.0
    sw.profile_reset()
    sw.profile_enable(True)
    for _ in range(reps):
        _run_once(sw, chars, offs, docs, n, nd, perm, boff, ws, stream)
    torch.cuda.synchronize()
    total = sum(v[1] for v in sw.profile_read().values()) / reps
    sw.profile_enable(False)
    return {"workload": name, "config": best, "kernel_ms": total, "trials": trials,
            "when": time.strftime("%Y-%m-%d %H:%M:%S")}


def _plan_ms(sw, torch, cfg, words, ref, runs: int = 10) -> float:
    chars, offs, docs, n, nd, perm, boff, stream = words
    sw.set_config(**cfg)
    plan = sw.Plan(n, nd, stream=stream)
    try:
        for _ in range(2):
            plan.run(chars, offs, docs, nd, n, perm, boff)
        plan.status()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(runs):
            plan.run(chars, offs, docs, nd, n, perm, boff)
        e1.record(stream)
        torch.cuda.synchronize()
        plan.status()
        if not (torch.equal(perm, ref[0]) and torch.equal(boff, ref[1])):
            raise RuntimeError("config %s changed the result" % (cfg,))
        return e0.elapsed_time(e1) / runs
    finally:
        plan.close()


def refine_on_plan(wl, cfg: dict, rounds: int = 3, log=print, variants: bool = True) -> dict:
    """Second stage: per class, the variant with the lowest median plan time;
    then the launch-order flags: whether each class's short-segment sort goes
    before its chunk sort (FLAG_PACKED_FIRST) and whether the segment
    scheduling runs beside the scatter (FLAG_SCHEDULE_BESIDE_SCATTER), every
    combination timed; then, with those, the 24 enqueue orders of the
    classes.  With variants=False only the flags and the order are timed."""
    import torch
    import paper_1411_5283_amd as sw

    dev = torch.device("cuda", torch.cuda.current_device())
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    chars, offs, docs = sw.device_words(wl, dev)
    n, nd = wl.n, wl.n_docs
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    boff = torch.empty(nd * 34, dtype=torch.int32, device=dev)
    words = (chars, offs, docs, n, nd, perm, boff, stream)
    best = {"chunk": list(cfg["chunk"]), "variant": list(cfg["variant"]), "flags": int(cfg.get("flags", 0))}
    sw.set_config(**best)
    plan = sw.Plan(n, nd, stream=stream)
    plan.run(chars, offs, docs, nd, n, perm, boff)
    plan.status()
    plan.close()
    ref = (perm.clone(), boff.clone())
    trials = []
    for c in range(NUM_CLASSES if variants else 0):
        times = {v: [] for v in range(sw.num_variants(c))}
        for _ in range(rounds):
            for v in times:
                trial = dict(best, variant=list(best["variant"]))
                trial["variant"][c] = v
                times[v].append(_plan_ms(sw, torch, trial, words, ref))
        med = {v: float(np.median(t)) for v, t in times.items()}
        for v, m in med.items():
            trials.append({"class": c, "variant": v, "plan_ms": m})
            log("plan: class %d variant %d: %.4f ms (median of %d)" % (c, v, m, rounds))
        bv = min(med, key=med.get)
        if med[bv] < 0.995 * med[best["variant"][c]]:
            best["variant"][c] = bv
    tunable = (sw.FLAG_PACKED_FIRST, sw.FLAG_SCHEDULE_BESIDE_SCATTER)
    combos = [sum(f for k, f in enumerate(tunable) if (m >> k) & 1) for m in range(1 << len(tunable))]
    order_bits = best["flags"] & sw.FLAG_ORDER_MASK
    times = {f: [] for f in combos}
    for _ in range(rounds):
        for f in times:
            times[f].append(_plan_ms(sw, torch, dict(best, flags=f | order_bits), words, ref))
    med = {f: float(np.median(t)) for f, t in times.items()}
    flag_trials = [{"flags": f, "plan_ms": m} for f, m in med.items()]
    for f, m in med.items():
        log("plan: flags %d: %.4f ms (median of %d)" % (f, m, rounds))
    bf = min(med, key=med.get)
    cur = best["flags"] & ~sw.FLAG_ORDER_MASK
    if med[bf] < 0.995 * med.get(cur, float("inf")):
        cur = bf
    order = (best["flags"] & sw.FLAG_ORDER_MASK) >> sw.FLAG_ORDER_SHIFT
    # then the classes' enqueue order, with those flags: the 24 orders of
    # classes 0-3 with class 4 (lengths 25-32, rare in text) last
    import itertools
    perms = list(itertools.permutations(range(NUM_CLASSES)))
    times = {perms.index(p + (NUM_CLASSES - 1,)): [] for p in itertools.permutations(range(NUM_CLASSES - 1))}
    for _ in range(rounds):
        for k in times:
            times[k].append(_plan_ms(sw, torch, dict(best, flags=cur | (k << sw.FLAG_ORDER_SHIFT)), words, ref))
    med = {k: float(np.median(t)) for k, t in times.items()}
    order_trials = [{"order": k, "plan_ms": m} for k, m in med.items()]
    log("plan: class orders: " + ", ".join("%d: %.4f" % (k, m) for k, m in med.items()))
    bk = min(med, key=med.get)
    if med[bk] < 0.995 * med[order]:
        order = bk
    best["flags"] = cur | (order << sw.FLAG_ORDER_SHIFT)
    sw.set_config(**best)
    final = float(np.median([_plan_ms(sw, torch, best, words, ref) for _ in range(rounds)]))
    out = {"config": best, "plan_ms": final, "flag_trials": flag_trials, "order_trials": order_trials}
    if variants:
        out["plan_trials"] = trials
    return out


def load_cache(path: str = CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save(result: dict, path: str = CACHE) -> None:
    cache = load_cache(path)
    cache.setdefault(device_key(), {})[result["workload"]] = result
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(workload: str, path: str = CACHE) -> dict | None:
    """Set the library's config to the cached best for this device and workload."""
    import paper_1411_5283_amd as sw
    entry = load_cache(path).get(device_key(), {}).get(workload)
    if not entry:
        return None
    cfg = entry["config"]
    return sw.set_config(chunk=cfg["chunk"], variant=cfg["variant"], flags=int(cfg.get("flags", 0)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--out", default=CACHE)
    ap.add_argument("--plan-only", action="store_true",
                    help="only the second stage, starting from the cached configuration")
    ap.add_argument("--plan-rounds", type=int, default=3, help="interleaved timing rounds per variant")
    ap.add_argument("--order-only", action="store_true",
                    help="with --plan-only: keep the cached variants, time only the launch-order flags")
    ap.add_argument("--chunk", type=int, default=None,
                    help="a workload that fixes the chunk size (the 250k-word list: 1024): tune the rest")
    args = ap.parse_args()
    from . import wordgen
    cfg = int(args.workload.lstrip("c"))
    wl = wordgen.config(cfg, args.scale)
    say = lambda *a: print(*a, flush=True)
    print("tuning on %s (%d words, %d documents)" % (args.workload, wl.n, wl.n_docs), flush=True)
    if args.plan_only:
        res = load_cache(args.out).get(device_key(), {}).get(args.workload)
        if not res:
            raise SystemExit("no cached configuration for %s" % args.workload)
    else:
        res = tune(wl, args.workload, reps=args.reps, chunks=(args.chunk,) if args.chunk else CHUNKS, log=say)
    res.update(refine_on_plan(wl, res["config"], rounds=args.plan_rounds, log=say,
                              variants=not (args.plan_only and args.order_only)))
    save(res, args.out)
    print(json.dumps({"workload": res["workload"], "config": res["config"], "kernel_ms": res["kernel_ms"],
                      "plan_ms": res["plan_ms"]}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
