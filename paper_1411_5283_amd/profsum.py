"""Summaries of rocprofv3 output for profiles/ (post-processing only).

    python -m paper_1411_5283_amd.profsum stats <kernel_stats.csv> "<command>" <out.txt>
    python -m paper_1411_5283_amd.profsum traffic <workload> <fetch.csv> <write.csv> <copy_fetch.csv> \
        <copy_write.csv> <bench.json> <out.json> [<text_fetch.csv> <text_write.csv>] [--outdir <dir>]
    python -m paper_1411_5283_amd.profsum valu <workload> <pmc_a.csv>,<pmc_b.csv> <bench.json> <out.json> \
        [--outdir <dir>]
    python -m paper_1411_5283_amd.profsum timeline <kernel_trace.csv> "<command>" <out.txt> [<step>]

--outdir names the folder the counter runs wrote to (it appears in the
commands each summary records); --extra "<args>" adds bench arguments to
those commands (e.g. a merge choice), and --tag names the runs' folders when
it is not the workload.

``traffic`` averages FETCH_SIZE and WRITE_SIZE (KiB per dispatch) per kernel
family and scales them by what the same counters read for a plain 1 GiB
device copy (``bench.py --copy-calibration``), so that the result is HBM
bytes per launch.  The sort's kernels come from a run without the text steps
(a run that writes text also keeps the sorted keys in the last merge level,
which changes that level's traffic); the text kernels, found only in the
second pair, from a run with them.

``timeline`` splits a ``rocprofv3 --kernel-trace`` record into passes (each
begins with ``k_begin``) and lists, for one pass (``<step>``, an index into
the passes, default -5: a timed plan replay before the eager profiling step
and the checks of a ``--steps 3 --profile-steps 1`` run), each kernel
family's first start, last end, busy time, launches and hardware queues,
relative to the pass's start.

``valu`` averages the SQ counters of two runs (VALU and LDS instructions
issued, the cycles waves spent in them, lane-cycles, LDS bank conflicts,
waves, busy cycles) per dispatch and kernel family.  Every value is summed
over the GPU's 8 XCDs and their shader engines; GRBM_GUI_ACTIVE too, so the
dispatch's clock count is that counter / 8.
"""
from __future__ import annotations

import collections
import csv
import json
import re
import sys

COPY_BYTES = 1 << 30
BENCH = ("python3 bench.py --workload {w} --serial --steps 1 --warmup 1 --profile-steps 1 --no-plain "
         "--no-cpu-baseline --no-check")
SQ_COUNTERS = ("SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_INSTS_LDS SQ_ACTIVE_INST_LDS SQ_LDS_BANK_CONFLICT SQ_WAVES "
               "SQ_BUSY_CYCLES SQ_INSTS_SALU GRBM_GUI_ACTIVE",
               "SQ_THREAD_CYCLES_VALU SQ_LDS_IDX_ACTIVE SQ_WAVE_CYCLES SQ_WAIT_INST_LDS SQ_ACTIVE_INST_VALU2 "
               "GRBM_GUI_ACTIVE")


def _bench_cmd(w: str, extra: str) -> str:
    return BENCH.format(w=w) + (" " + extra if extra else "")


def traffic_commands(w: str, d: str, extra: str = "", tag: str = "", text: bool = True) -> list:
    """The runs a traffic summary is made from; d: the folder they wrote to."""
    b, t = _bench_cmd(w, extra), tag or w
    cmds = [
        "rocprofv3 --pmc FETCH_SIZE --output-format csv -d %s/f_%s -o f -- %s --no-text" % (d, t, b),
        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d %s/w_%s -o w -- %s --no-text" % (d, t, b),
    ]
    if text:
        cmds += ["rocprofv3 --pmc FETCH_SIZE --output-format csv -d %s/ft_%s -o f -- %s" % (d, t, b),
                 "rocprofv3 --pmc WRITE_SIZE --output-format csv -d %s/wt_%s -o w -- %s" % (d, t, b)]
    return cmds + [
        "rocprofv3 --pmc FETCH_SIZE --output-format csv -d %s/cf -o cf -- python3 bench.py --copy-calibration" % d,
        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d %s/cw -o cw -- python3 bench.py --copy-calibration" % d,
    ]


def valu_commands(w: str, d: str, extra: str = "", tag: str = "") -> list:
    return ["rocprofv3 --pmc %s --output-format csv -d %s/sq%d_%s -o s -- %s --no-text" % (
        c, d, i, tag or w, _bench_cmd(w, extra)) for i, c in enumerate(SQ_COUNTERS)]


def stats(src: str, cmd: str, out: str) -> None:
    rows = list(csv.DictReader(open(src)))
    lines = ["# rocprofv3 kernel statistics", "#",
             "# command (run from the repository root on one MI355X):", "#   " + cmd, "#",
             "# %-64s %6s %14s %12s %7s" % ("kernel", "calls", "total_ns", "avg_ns", "pct")]
    for r in rows:
        lines.append("  %-64s %6s %14s %12.0f %7.2f" % (r["Name"][:64], r["Calls"], r["TotalDurationNs"],
                                                       float(r["AverageNs"]), float(r["Percentage"])))
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def timeline(src: str, cmd: str, out: str, step: int = -5) -> None:
    rows = sorted(csv.DictReader(open(src)), key=lambda r: int(r["Start_Timestamp"]))
    passes, cur = [], None
    for r in rows:
        if re.match(r"(?:void )?sw::k_begin\b", r["Kernel_Name"]):
            cur = []
            passes.append(cur)
        if cur is not None:
            cur.append(r)
    ps = passes[step]
    t0 = int(ps[0]["Start_Timestamp"])
    fams = collections.OrderedDict()
    for r in ps:
        f = _family(r["Kernel_Name"].split("(")[0]) or r["Kernel_Name"][:24]
        a, b = (int(r["Start_Timestamp"]) - t0) / 1e3, (int(r["End_Timestamp"]) - t0) / 1e3
        g = fams.setdefault(f, [a, b, 0.0, 0, set()])
        g[0], g[1] = min(g[0], a), max(g[1], b)
        g[2] += b - a
        g[3] += 1
        g[4].add(r["Queue_Id"])
    span = (max(int(r["End_Timestamp"]) for r in ps) - t0) / 1e3
    lines = ["# rocprofv3 kernel trace: one pass of the plan, kernel families in order of first start", "#",
             "# command (run from the repository root on one MI355X):", "#   " + cmd, "#",
             "# pass %d of %d (%d kernels, %.1f us from the first start to the last end, under the profiler)"
             % (step % len(passes), len(passes), len(ps), span), "#",
             "# %-18s %10s %10s %10s %6s  %s" % ("family", "first_us", "last_us", "busy_us", "calls", "queues")]
    for f, g in fams.items():
        lines.append("  %-18s %10.1f %10.1f %10.1f %6d  %s" % (f, g[0], g[1], g[2], g[3], ",".join(sorted(g[4]))))
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def _family(kernel: str) -> str | None:
    """Kernel name -> the bench's family name: the per-class kernels (chunk
    sorts and merges, whose first template argument is the key lanes, 0-4 for
    classes 0-4) get the class as a suffix, every other kernel its own name."""
    m = re.match(r"(?:void )?sw::k_(\w+?)(?:<(\d+)|[<(]|$)", kernel)
    if not m:
        return None
    name = m.group(1)
    if name in ("sort_tiles", "sort_packed", "merge", "merge4w"):
        nl = int(m.group(2)) if m.group(2) else -1
        return "%s_c%d" % ("merge" if name == "merge4w" else name, nl) if 0 <= nl <= 4 else None
    return name


def _per_dispatch(path: str, counter: str) -> dict:
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            agg[r["Kernel_Name"].split("(")[0].replace("void ", "")].append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in agg.items()}


def _bench_line(bench_json: str) -> dict:
    with open(bench_json) as fh:
        return json.loads(fh.read().strip().splitlines()[-1])


def _tiles(b: dict) -> dict:
    c = b["config"]
    return {"chunk": c.get("chunk"), "variant": c.get("variant"), "merge": c.get("merge")}


def traffic(workload: str, fetch: str, write: str, cfetch: str, cwrite: str, bench_json: str, out: str,
            text_fetch: str | None = None, text_write: str | None = None, outdir: str = "out",
            extra: str = "", tag: str = "") -> None:
    f = _per_dispatch(fetch, "FETCH_SIZE")
    w = _per_dispatch(write, "WRITE_SIZE")
    if text_fetch and text_write:
        fams = {_family(k) for k in f}
        tf = _per_dispatch(text_fetch, "FETCH_SIZE")
        tw = _per_dispatch(text_write, "WRITE_SIZE")
        for k, v in tf.items():
            if _family(k) not in fams and k in tw:
                f[k] = v
                w[k] = tw[k]
    cf = _per_dispatch(cfetch, "FETCH_SIZE")["__amd_rocclr_copyBuffer"][0]
    cw = _per_dispatch(cwrite, "WRITE_SIZE")["__amd_rocclr_copyBuffer"][0]
    fs, wsc = COPY_BYTES / 1024 / cf, COPY_BYTES / 1024 / cw
    b = _bench_line(bench_json)
    kern = {}
    for k, (fk, nd) in f.items():
        fam = _family(k)
        if fam is None or k not in w:
            continue
        wk = w[k][0]
        kern[fam] = {"kernel": k, "dispatches": nd, "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk,
                     "bytes_per_launch": fk * 1024 * fs + wk * 1024 * wsc}
    res = {"source_hash": b["kernel_source"], "workload": b["config"]["workload"] + " (bench.py --serial)",
           "tiles": _tiles(b), "fetch_scale": fs, "write_scale": wsc,
           "calibration": "plain device copy of 1 GiB (__amd_rocclr_copyBuffer): FETCH_SIZE %.0f KiB, "
                          "WRITE_SIZE %.0f KiB per dispatch" % (cf, cw),
           "commands": traffic_commands(workload, outdir, extra, tag, bool(text_fetch and text_write)),
           "kernels": kern}
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1, sort_keys=True)


def valu(workload: str, pmcs: str, bench_json: str, out: str, outdir: str = "out", extra: str = "",
         tag: str = "") -> None:
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for pmc in pmcs.split(","):
        for r in csv.DictReader(open(pmc)):
            k = r["Kernel_Name"].split("(")[0].replace("void ", "")
            agg[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
    b = _bench_line(bench_json)
    kern = {}
    for k, cs in agg.items():
        fam = _family(k)
        if fam is None:
            continue
        row = {"kernel": k, "dispatches": len(cs["SQ_INSTS_VALU"]) if "SQ_INSTS_VALU" in cs else None}
        for name, vals in cs.items():
            row[name + "_per_dispatch"] = sum(vals) / len(vals)
        kern[fam] = row
    res = {"source_hash": b["kernel_source"], "workload": b["config"]["workload"] + " (bench.py --serial)",
           "tiles": _tiles(b), "commands": valu_commands(workload, outdir, extra, tag), "kernels": kern,
           "note": "SQ_INSTS_VALU counts wave instructions (each up to 64 lanes); SQ_ACTIVE_INST_VALU and "
                   "SQ_ACTIVE_INST_LDS are quad-cycles summed over waves; every value is summed over the "
                   "shader engines and the 8 XCDs (GRBM_GUI_ACTIVE / 8 = the dispatch's clocks)"}
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    argv = list(sys.argv[1:])
    opts = {"--outdir": "out", "--extra": "", "--tag": ""}
    for name in opts:   # the recorded commands: runs' folder, extra bench arguments, folder tag
        if name in argv:
            k = argv.index(name)
            opts[name] = argv[k + 1]
            del argv[k:k + 2]
    kw = {"outdir": opts["--outdir"], "extra": opts["--extra"], "tag": opts["--tag"]}
    if argv[0] == "stats":
        stats(*argv[1:4])
    elif argv[0] == "traffic":
        traffic(*argv[1:10], **kw)
    elif argv[0] == "valu":
        valu(*argv[1:5], **kw)
    elif argv[0] == "timeline":
        timeline(argv[1], argv[2], argv[3], *([int(argv[4])] if len(argv) > 4 else []))
    else:
        raise SystemExit(__doc__)
