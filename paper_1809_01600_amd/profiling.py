"""Profiling helpers: a plain device copy of known size (to calibrate the HBM byte counters) and a
summarizer of rocprofv3 CSV output.

  python -m paper_1809_01600_amd.profiling copy --mib 1024 --reps 5
  python -m paper_1809_01600_amd.profiling summarize <rocprofv3 output dir> [--kernel NAME]
  python -m paper_1809_01600_amd.profiling report --name NAME --key KEY --kernel K \
      --trace DIR --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR \
      --alg-bytes B --command "..." [--counter-command "..."]
      (writes profiles/NAME.txt and profiles/traffic.json)
"""

from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sys


def run_copy(mib: int, reps: int) -> None:
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "reps": reps}))


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def summarize(d: str, kernel: str = "") -> dict:
    out = {}
    stats = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    if stats:
        rows = _rows(stats[0])
        out["kernel_stats"] = [
            {"name": r.get("Name", "")[:120], "calls": int(r.get("Calls", 0)),
             "avg_ns": float(r.get("AverageNs", 0)), "total_ns": float(r.get("TotalDurationNs", 0)),
             "pct": float(r.get("Percentage", 0))}
            for r in rows if kernel in r.get("Name", "")]
    trace = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)
    if trace:
        rows = [r for r in _rows(trace[0]) if kernel in r.get("Kernel_Name", "")]
        if rows:
            starts = sorted(int(r["Start_Timestamp"]) for r in rows)
            ends = sorted(int(r["End_Timestamp"]) for r in rows)
            durs = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows]
            gaps = [starts[i + 1] - ends[i] for i in range(len(starts) - 1)]
            gaps.sort()
            out["trace"] = {"dispatches": len(rows), "avg_ns": sum(durs) / len(durs),
                            "min_ns": min(durs), "max_ns": max(durs),
                            "median_gap_ns": gaps[len(gaps) // 2] if gaps else None}
    counters = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if counters:
        rows = _rows(counters[0])
        agg = {}
        for r in rows:
            name = r.get("Kernel_Name", "")
            if kernel and kernel not in name:
                continue
            cname = r.get("Counter_Name", "")
            key = (name[:120], cname)
            agg.setdefault(key, []).append(float(r.get("Counter_Value", 0)))
        out["counters"] = [{"kernel": k[0], "counter": k[1], "dispatches": len(v),
                            "mean_per_dispatch": sum(v) / len(v)} for k, v in agg.items()]
    return out


def _counter_mean(d: str, kernel: str, counter: str) -> float:
    for c in summarize(d, kernel).get("counters", []):
        if c["counter"] == counter:
            return c["mean_per_dispatch"]
    raise KeyError("%s not found for %s in %s" % (counter, kernel, d))


def report(args) -> None:
    """Summary text of one kernel's trace and counters, with the copy calibration, and the
    traffic record that bench.py reports."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import bench
    copy_bytes = args.copy_mib * (1 << 20)
    cf = _counter_mean(args.copy_fetch, "copyBuffer", "FETCH_SIZE")
    cw = _counter_mean(args.copy_write, "copyBuffer", "WRITE_SIZE")
    f_scale = copy_bytes / (cf * 1024.0)
    w_scale = copy_bytes / (cw * 1024.0)
    kf = _counter_mean(args.fetch, args.kernel, "FETCH_SIZE")
    kw = _counter_mean(args.write, args.kernel, "WRITE_SIZE")
    fetch_b = kf * 1024.0 * f_scale
    write_b = kw * 1024.0 * w_scale
    tr = summarize(args.trace, args.kernel)
    stats = tr.get("kernel_stats", [])
    lines = []
    lines.append("rocprofv3 summary: %s" % args.name)
    lines.append("command (trace): %s" % args.command)
    lines.append("counters: %s" % (args.counter_command or
                                   "same program under rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE"))
    lines.append("calibration: python3 -m paper_1809_01600_amd.profiling copy --mib %d --reps 5 under"
                 " the same two counters" % args.copy_mib)
    lines.append("")
    lines.append("kernel stats (--kernel-trace --stats):")
    for k in stats:
        lines.append("  %-70s calls %6d  avg %10.1f ns  total %12.0f ns  %5.1f%%" % (
            k["name"][:70], k["calls"], k["avg_ns"], k["total_ns"], k["pct"]))
    if "trace" in tr:
        t = tr["trace"]
        lines.append("  trace: %d dispatches, avg %.1f ns, min %d, max %d, median gap %s ns" % (
            t["dispatches"], t["avg_ns"], t["min_ns"], t["max_ns"], t["median_gap_ns"]))
    lines.append("")
    lines.append("copy calibration (%d MiB read + written per dispatch): FETCH_SIZE %.1f KiB -> x%.4f,"
                 " WRITE_SIZE %.1f KiB -> x%.4f" % (args.copy_mib, cf, f_scale, cw, w_scale))
    lines.append("step kernel per dispatch: FETCH_SIZE %.1f KiB -> %.3f MB, WRITE_SIZE %.1f KiB -> %.3f MB"
                 % (kf, fetch_b / 1e6, kw, write_b / 1e6))
    lines.append("measured HBM-side traffic per launch: %.3f MB; algorithmic: %.3f MB (ratio %.3f)" % (
        (fetch_b + write_b) / 1e6, args.alg_bytes / 1e6, (fetch_b + write_b) / args.alg_bytes))
    if stats:
        avg = stats[0]["avg_ns"]
        lines.append("achieved (algorithmic bytes / avg duration): %.1f GB/s = %.1f%% of 8000 GB/s" % (
            args.alg_bytes / avg, 100.0 * args.alg_bytes / avg / 8000.0))
    os.makedirs(os.path.join(root, "profiles"), exist_ok=True)
    with open(os.path.join(root, "profiles", args.name + ".txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    tpath = os.path.join(root, "profiles", "traffic.json")
    data = {}
    if os.path.exists(tpath):
        with open(tpath) as f:
            data = json.load(f)
    data[args.key] = {"kernel_hash": bench.kernel_hash(), "bytes_per_launch": round(fetch_b + write_b),
                      "fetch_bytes": round(fetch_b), "write_bytes": round(write_b),
                      "avg_ns": stats[0]["avg_ns"] if stats else None, "profile": args.name + ".txt"}
    with open(tpath, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print("\n".join(lines))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=1024)
    c.add_argument("--reps", type=int, default=5)
    s = sub.add_parser("summarize")
    s.add_argument("dir")
    s.add_argument("--kernel", default="")
    r = sub.add_parser("report")
    for a in ("name", "key", "kernel", "trace", "fetch", "write", "copy_fetch", "copy_write",
              "command"):
        r.add_argument("--" + a.replace("_", "-"), required=True)
    r.add_argument("--alg-bytes", type=float, required=True)
    r.add_argument("--copy-mib", type=int, default=1024)
    r.add_argument("--counter-command", default="")
    args = ap.parse_args(argv)
    if args.cmd == "copy":
        run_copy(args.mib, args.reps)
    elif args.cmd == "report":
        report(args)
    else:
        print(json.dumps(summarize(args.dir, args.kernel), indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
