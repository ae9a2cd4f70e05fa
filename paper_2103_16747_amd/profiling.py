"""Summaries of rocprofv3 CSV output for the indentation kernels.

    python -m paper_2103_16747_amd.profiling stats  <rocprof dir> [--kernel REGEX]
    python -m paper_2103_16747_amd.profiling traffic <fetch dir> <write dir> --copy-bytes N [--kernel REGEX]
    python -m paper_2103_16747_amd.profiling counters <pmc dir> --kernel REGEX
    python -m paper_2103_16747_amd.profiling traffic-json <fetch dir> <write dir> --copy-bytes N --out FILE

`stats` reads a --kernel-trace --stats run (kernel_stats.csv / kernel_trace.csv)
and prints per-kernel calls and durations. `traffic` reads two --pmc runs, one
with FETCH_SIZE and one with WRITE_SIZE (KiB per dispatch), and converts them
to bytes with the ratio the same counters give for a plain device copy of
N bytes in the same process (the benchmark's --copy-mb option), reporting the
per-dispatch HBM traffic of the matching kernels.
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
import re
import statistics
import sys


def _find(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def kernel_stats(d, pattern=None):
    rows = list(csv.DictReader(open(_find(d, "kernel_stats.csv"))))
    out = []
    for r in rows:
        if pattern and not re.search(pattern, r["Name"]):
            continue
        out.append({"name": r["Name"], "calls": int(r["Calls"]), "avg_us": float(r["AverageNs"]) / 1e3,
                    "min_us": float(r["MinNs"]) / 1e3, "max_us": float(r["MaxNs"]) / 1e3,
                    "total_ms": float(r["TotalDurationNs"]) / 1e6, "pct": float(r["Percentage"])})
    return out


def busy_kernel_stats(d, pattern, floor_us):
    """Durations of dispatches of `pattern` longer than floor_us (dispatches
    whose jobs were all in other solver phases exit at once and are left
    out), from kernel_trace.csv."""
    durs = []
    for r in csv.DictReader(open(_find(d, "kernel_trace.csv"))):
        if re.search(pattern, r["Kernel_Name"]):
            us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            if us >= floor_us:
                durs.append(us)
    if not durs:
        return None
    return {"dispatches": len(durs), "avg_us": statistics.mean(durs), "median_us": statistics.median(durs)}


def counters(d):
    per = {}
    for r in csv.DictReader(open(_find(d, "counter_collection.csv"))):
        per.setdefault(r["Kernel_Name"], {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return per


def traffic(fetch_dir, write_dir, copy_bytes, pattern, copy_pattern=r"copy|elementwise|Copy"):
    """Per-dispatch HBM bytes of the kernels matching `pattern`: the mean of
    FETCH_SIZE and of WRITE_SIZE over all their dispatches, each scaled by
    copy_bytes over what the same counter read for the largest copy dispatch
    (the calibration copy)."""
    fc, wc = counters(fetch_dir), counters(write_dir)

    def pick(cs, name, pat):
        return [v for k, m in cs.items() if re.search(pat, k) for v in m.get(name, [])]

    cf = pick(fc, "FETCH_SIZE", copy_pattern)
    cw = pick(wc, "WRITE_SIZE", copy_pattern)
    if not cf or not cw:
        raise RuntimeError("no copy-kernel counters found")
    f_scale = copy_bytes / (max(cf) * 1024.0)
    w_scale = copy_bytes / (max(cw) * 1024.0)
    kf = pick(fc, "FETCH_SIZE", pattern)
    kw = pick(wc, "WRITE_SIZE", pattern)
    if not kf or not kw:
        raise RuntimeError("no counters for " + pattern)
    fetch = statistics.mean(kf) * 1024.0 * f_scale
    write = statistics.mean(kw) * 1024.0 * w_scale
    return {"copy_fetch_KiB": max(cf), "copy_write_KiB": max(cw), "fetch_scale": f_scale, "write_scale": w_scale,
            "dispatches_fetch": len(kf), "dispatches_write": len(kw),
            "fetch_bytes_per_dispatch": fetch, "write_bytes_per_dispatch": write,
            "traffic_bytes_per_dispatch": fetch + write}


def counter_means(d, pattern, busy_floor_us=0.0):
    """Per-dispatch means of every counter of a --pmc run for the kernels
    matching `pattern`, with the number of dispatches and their mean
    duration (us, from the dispatch timestamps); with busy_floor_us > 0,
    over the dispatches that lasted longer than that only."""
    per, dur = {}, {}
    for r in csv.DictReader(open(_find(d, "counter_collection.csv"))):
        if not re.search(pattern, r["Kernel_Name"]):
            continue
        i = r["Dispatch_Id"]
        c = per.setdefault(i, {})
        c[r["Counter_Name"]] = c.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        dur[i] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    sel = [i for i in dur if dur[i] > busy_floor_us]
    if not sel:
        raise RuntimeError("no counters for " + pattern)
    names = sorted({k for i in sel for k in per[i]})
    return {"dispatches": len(sel), "mean_duration_us": statistics.mean(dur[i] for i in sel),
            "per_dispatch": {k: sum(per[i].get(k, 0.0) for i in sel) / len(sel) for k in names}}


def kernel_source_hash(text=None):
    """SHA-256 of the device source with comments and blank lines removed;
    traffic figures are valid only for the kernels they were taken on."""
    import hashlib
    if text is None:
        here = os.path.dirname(os.path.abspath(__file__))
        with open(os.path.join(here, "csrc", "fem_kernels.h")) as f:
            text = f.read()
    code = []
    for line in text.splitlines():
        line = line.split("//", 1)[0].rstrip()
        if line.strip():
            code.append(line)
    return hashlib.sha256("\n".join(code).encode()).hexdigest()


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    a.add_argument("--kernel", default=None)
    a.add_argument("--busy-floor-us", type=float, default=0.0)
    b = sub.add_parser("traffic")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("--copy-bytes", type=float, required=True)
    b.add_argument("--kernel", required=True)
    b.add_argument("--json", default=None, help="also write the result here, with the kernel source hash")
    d = sub.add_parser("traffic-json", help="tile and node kernel traffic into one file for bench.py")
    d.add_argument("fetch_dir")
    d.add_argument("write_dir")
    d.add_argument("--copy-bytes", type=float, required=True)
    d.add_argument("--groups", type=int, default=1, help="job groups per round of the profiled run")
    d.add_argument("--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("--kernel", required=True)
    c.add_argument("--busy-floor-us", type=float, default=0.0)
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        for r in kernel_stats(args.dir, args.kernel):
            print(f"{r['name'][:72]:72s} calls={r['calls']:7d} avg={r['avg_us']:9.2f}us min={r['min_us']:8.2f}us "
                  f"max={r['max_us']:9.2f}us total={r['total_ms']:9.2f}ms {r['pct']:5.1f}%")
        if args.kernel and args.busy_floor_us > 0:
            print("busy dispatches:", busy_kernel_stats(args.dir, args.kernel, args.busy_floor_us))
    elif args.cmd == "counters":
        r = counter_means(args.dir, args.kernel, args.busy_floor_us)
        print(f"dispatches {r['dispatches']}  mean duration {r['mean_duration_us']:.2f} us")
        for k, v in r["per_dispatch"].items():
            print(f"  {k:28s} {v:.4e} per dispatch")
    elif args.cmd == "traffic-json":
        import json
        rec = {"kernel_source_sha256": kernel_source_hash(), "groups": args.groups}
        for key, pat in (("tile", r"k_tile<float, 0, false>"), ("node", r"k_node<float, false>")):
            t = traffic(args.fetch_dir, args.write_dir, args.copy_bytes, pat)
            rec[f"{key}_bytes_per_dispatch"] = t["traffic_bytes_per_dispatch"]
            rec[f"{key}_fetch_bytes_per_dispatch"] = t["fetch_bytes_per_dispatch"]
            rec[f"{key}_write_bytes_per_dispatch"] = t["write_bytes_per_dispatch"]
            rec[f"{key}_dispatches"] = t["dispatches_fetch"]
            rec["fetch_scale"], rec["write_scale"] = t["fetch_scale"], t["write_scale"]
            print(f"{key}: {t['traffic_bytes_per_dispatch'] / 1e6:.1f} MB per dispatch "
                  f"({t['fetch_bytes_per_dispatch'] / 1e6:.1f} fetched, {t['write_bytes_per_dispatch'] / 1e6:.1f} written, "
                  f"{t['dispatches_fetch']} dispatches)")
        with open(args.out, "w") as f:
            json.dump(rec, f, indent=1)
    else:
        t = traffic(args.fetch_dir, args.write_dir, args.copy_bytes, args.kernel)
        for k, v in t.items():
            print(f"{k}: {v}")
        if args.json:
            import json
            t["kernel"] = args.kernel
            t["kernel_source_sha256"] = kernel_source_hash()
            with open(args.json, "w") as f:
                json.dump(t, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
