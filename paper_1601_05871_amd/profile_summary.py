"""Summaries of rocprofv3 output for the library's kernels.

    python -m paper_1601_05871_amd.profile_summary stats <dir-with-*_kernel_stats.csv>
    python -m paper_1601_05871_amd.profile_summary pmc <results.db> [--match NAME]
    python -m paper_1601_05871_amd.profile_summary source-hash

``stats`` prints the per-kernel table of ``rocprofv3 --kernel-trace --stats
--output-format csv``; ``pmc`` sums each counter of ``rocprofv3 --pmc`` over
the dispatches of each kernel (FETCH_SIZE / WRITE_SIZE are in KiB);
``source-hash`` prints the hash of the trailing-update kernel sources that a
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
    s = name.split("(")[0] if "(" in name and "<" not in name.split("(")[0][-1:] else name
    s = s.replace("void ", "").replace("flame::", "")
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


def main() -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("path")
    a.add_argument("--top", type=int, default=25)
    b = sub.add_parser("pmc")
    b.add_argument("db")
    b.add_argument("--match")
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
    else:
        print(gemm_source_hash())


if __name__ == "__main__":
    main()
