"""Summaries of rocprofv3 output for the library's kernels.

    python -m paper_1601_05871_amd.profile_summary stats <dir-with-*_kernel_stats.csv>
    python -m paper_1601_05871_amd.profile_summary pmc <results.db> [--match NAME]
    python -m paper_1601_05871_amd.profile_summary busy <dir-with-*_kernel_trace.csv> --match NAME
    python -m paper_1601_05871_amd.profile_summary source-hash

``stats`` prints the per-kernel table of ``rocprofv3 --kernel-trace --stats
--output-format csv``; ``pmc`` sums each counter of ``rocprofv3 --pmc`` over
the dispatches of each kernel (FETCH_SIZE / WRITE_SIZE are in KiB);
``busy`` reads the dispatch intervals of ``rocprofv3 --kernel-trace
--output-format csv`` and prints, for the kernels whose name contains NAME,
the number of dispatches, the sum of their durations, the length of the union
of their intervals (dispatches that overlap count once) and the whole traced
span; ``source-hash`` prints the hash of the trailing-update kernel sources that a
traffic summary is tied to.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import sqlite3
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
GEMM_SOURCES = ("csrc/k_gemm.hip", "csrc/tile_map.h")


def gemm_source_hash() -> str:
    h = hashlib.sha256()
    for rel in GEMM_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short(name: str, width: int = 72) -> str:
    s = name
    if s.endswith(")"):  # drop the parameter list (the parenthesis matching the last one)
        depth = 0
        for i in range(len(s) - 1, -1, -1):
            depth += {")": 1, "(": -1}.get(s[i], 0)
            if depth == 0:
                s = s[:i]
                break
    s = s.replace("void ", "").replace("(anonymous namespace)::", "").replace("flame::", "")
    return s if len(s) <= width else s[:width - 3] + "..."


def stats(path: str, top: int = 25) -> list[dict]:
    files = glob.glob(os.path.join(path, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no *kernel_stats.csv under {path}")
    rows = []
    with open(files[0]) as f:
        for r in csv.DictReader(f):
            rows.append({"name": r["Name"], "calls": int(r["Calls"]), "total_ns": float(r["TotalDurationNs"]),
                         "avg_ns": float(r["AverageNs"]), "pct": float(r["Percentage"]),
                         "min_ns": float(r["MinNs"]), "max_ns": float(r["MaxNs"])})
    rows.sort(key=lambda r: -r["total_ns"])
    return rows[:top]


def pmc(db: str, match: str | None = None) -> dict:
    con = sqlite3.connect(db)
    cur = con.cursor()
    acc = defaultdict(lambda: defaultdict(float))
    disp = defaultdict(set)
    for d, k, c, v in cur.execute("select dispatch_id, kernel_name, counter_name, value from counters_collection"):
        if match and match not in k:
            continue
        acc[k][c] += float(v)
        disp[k].add(d)
    return {k: {"dispatches": len(disp[k]), **{c: v for c, v in cs.items()}} for k, cs in acc.items()}


def busy(path: str, match: str) -> dict:
    files = glob.glob(os.path.join(path, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no *kernel_trace.csv under {path}")
    iv = []
    lo, hi = None, None
    with open(files[0]) as f:
        for r in csv.DictReader(f):
            t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
            lo = t0 if lo is None else min(lo, t0)
            hi = t1 if hi is None else max(hi, t1)
            if match in r["Kernel_Name"]:
                iv.append((t0, t1))
    iv.sort()
    total = sum(b - a for a, b in iv)
    union, c0, c1 = 0, None, None
    for a, b in iv:
        if c1 is None or a > c1:
            if c1 is not None:
                union += c1 - c0
            c0, c1 = a, b
        else:
            c1 = max(c1, b)
    if c1 is not None:
        union += c1 - c0
    return {"dispatches": len(iv), "sum_ms": total / 1e6, "union_ms": union / 1e6,
            "avg_us": total / max(1, len(iv)) / 1e3, "span_ms": (hi - lo) / 1e6 if iv else 0.0}


def main() -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("path")
    a.add_argument("--top", type=int, default=25)
    b = sub.add_parser("pmc")
    b.add_argument("db")
    b.add_argument("--match")
    c = sub.add_parser("busy")
    c.add_argument("path")
    c.add_argument("--match", required=True)
    sub.add_parser("source-hash")
    args = ap.parse_args()
    if args.cmd == "stats":
        print(f"| kernel | calls | avg us | total ms | % |\n|---|---|---|---|---|")
        for r in stats(args.path, args.top):
            print(f"| `{short(r['name'])}` | {r['calls']} | {r['avg_ns'] / 1e3:.1f} | {r['total_ns'] / 1e6:.3f} | "
                  f"{r['pct']:.2f} |")
    elif args.cmd == "pmc":
        res = pmc(args.db, args.match)
        for k, cs in sorted(res.items(), key=lambda kv: -max(v for c, v in kv[1].items() if c != "dispatches")):
            nd = cs["dispatches"]
            vals = ", ".join(f"{c} total {v:.6g} (per dispatch {v / nd:.6g})" for c, v in cs.items()
                             if c != "dispatches")
            print(f"{short(k)} | dispatches {nd} | {vals}")
    elif args.cmd == "busy":
        r = busy(args.path, args.match)
        print(f"kernels matching `{args.match}`: {r['dispatches']} dispatches, summed duration {r['sum_ms']:.3f} ms "
              f"(average {r['avg_us']:.1f} us), union of intervals {r['union_ms']:.3f} ms, traced span "
              f"{r['span_ms']:.3f} ms")
    else:
        print(gemm_source_hash())


if __name__ == "__main__":
    main()
