#!/usr/bin/env python3
"""Benchmark of the blocked Cholesky A = U^T U (Fig. "dense-chol") on one
MI355X.

A step is one FP64 factorization of the n = 16384 SPD matrix A = B B^T + n I
(B ~ N(0,1), PCG64 seed), right-looking loop, block size 512 (256, then 128
for the last 8192 and 6144 columns), lookahead.
Each timed step factors its own pre-generated copy already resident in HBM,
so the timed region holds nothing but the K factorizations.  Prints one JSON
line with GFLOP/s (potrf flop count n^3/3 + n^2/2 + n/6), the live roofline of
the dominant kernel (the trailing SYRK/GEMM: its flops over the union of its
launch intervals, from per-launch HIP events), the mixed-precision time to
solution against the FP64 path at equal backward error for every
kappa x trail x nrhs cell, the batched factorization, and the CPU oracle's
rate on the host cores.

    python bench.py [--gpus 1] [--steps 5] [--warmup 2]
    python bench.py --table [--steps 2]     # the n x nb x variant x seed sweep
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GFLOP/s & %MFMA peak at n=16384, mixed vs FP64, equal backward err"
PEAK_F64_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
PEAK_F32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def potrf_flops(n: int) -> float:
    return float(n * (n + 1) * (2 * n + 1) // 6)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--nb", type=int, default=512)
    ap.add_argument("--variant", type=int, default=3)
    ap.add_argument("--lookahead", type=int, default=2)
    ap.add_argument("--graph", type=int, default=0)
    ap.add_argument("--no-trace", action="store_true",
                    help="time without the per-launch events (no roofline figures)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--kappas", default="1e2,1e4,1e6", help="condition numbers of the mixed-precision cells")
    ap.add_argument("--trails", default="f32,bf16", help="trailing-product precisions of the mixed cells")
    ap.add_argument("--nrhs", default="1,64", help="right-hand-side counts of the mixed cells")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--table", action="store_true",
                    help="instead of the default run: time every (n, nb, variant, seed) cell of the "
                         "single-matrix FP64 sweep and print a markdown table")
    ap.add_argument("--dag", action="store_true",
                    help="instead of the default run: the by-blocks task DAG (flame_factor_by_blocks) against "
                         "the default right-looking loop at each n of --table-ns, one JSON line per order")
    ap.add_argument("--ichol", action="store_true",
                    help="instead of the default run: level(k) incomplete Cholesky-by-blocks (flame_ichol_*) on "
                         "grid Laplacians, with the oracle's sequential incomplete factor timed beside it")
    ap.add_argument("--extensions", action="store_true",
                    help="instead of the default run: the complex Hermitian factorization (flame_factor, "
                         "complex128) and the LU without pivoting (flame_lu) at the orders of --ext-ns, with the "
                         "oracle's unblocked loops timed beside them at --ext-oracle-n")
    ap.add_argument("--ext-ns", default="2048,4096,8192")
    ap.add_argument("--ext-cases", default="complex,lu,qr",
                    help="with --extensions: qr alone runs only the QR case (for profiles)")
    ap.add_argument("--ext-oracle-n", type=int, default=1024)
    ap.add_argument("--table-ns", default="4096,8192,16384")
    ap.add_argument("--table-nbs", default="64,128,256")
    ap.add_argument("--table-seeds", default="0,1,2")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-extensions", action="store_true",
                    help="leave out the complex / LU / QR timings at n = 8192 of the default line")
    ap.add_argument("--batch", type=int, default=10000)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="one plain device copy of this many GiB before the timed region (a reference "
                         "kernel of known traffic for HBM counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the factorization of one matrix is measured on a single "
              "MI355X (no collectives in this build); run with --gpus 1", file=sys.stderr)
        return 2

    import torch
    import inputs
    import paper_1601_05871_amd as fl

    fl.lib()  # fails loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.table:
        return table_mode(args, dev, fl, inputs, torch)
    if args.dag:
        return dag_mode(args, dev, fl, inputs, torch)
    if args.ichol:
        return ichol_mode(args, dev, fl, inputs, torch)
    if args.extensions:
        return extensions_mode(args, dev, fl, inputs, torch)
    if args.copy_probe_gib > 0:
        words = int(args.copy_probe_gib * (1 << 30)) // 8
        src = torch.ones(words, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)  # a streaming kernel of its own name: reads and writes words * 8 bytes
        torch.cuda.synchronize()
        log(f"copy probe (neg kernel): {words * 8} bytes read, {words * 8} bytes written")
        del src, dst
    n, K, W = args.n, max(1, args.steps), max(0, args.warmup)
    log(f"generating A = B B^T + n I, n={n}, seed={args.seed}")
    P = inputs.spd_bbt_torch(n, args.seed, dev)  # pristine, column-major
    copies = [torch.empty_strided((n, n), (1, n), dtype=torch.float64, device=dev) for _ in range(K)]
    infos = torch.zeros(K, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def factor(M, info):
        return fl.factor(M, variant=args.variant, nb=args.nb, lookahead=args.lookahead, graph=args.graph, info=info)

    log(f"warmup x{W}")
    for _ in range(W):
        copies[0].copy_(P)
        factor(copies[0], infos[0:1])
    for c in copies:
        c.copy_(P)
    torch.cuda.synchronize()

    # ---- timed region: K factorizations, inputs resident in HBM -------------
    log(f"timing {K} factorizations")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(K):
        factor(copies[i], infos[i:i + 1])
    ev1.record(stream)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    ev_ms = ev0.elapsed_time(ev1)
    ms_per_step = ev_ms / K
    info_h = infos.cpu().numpy()
    if np.any(info_h != 0):
        log(f"factorization reported breakdown: {info_h}")
        return 1
    gflops = potrf_flops(n) / (ms_per_step * 1e-3) / 1e9
    log(f"{ms_per_step:.3f} ms/factorization = {gflops:.1f} GFLOP/s (wall {wall_ms / K:.3f} ms)")

    # ---- instrumented pass: the same K factorizations again (inputs restored
    # first) with HIP events around every kernel launch, on the stream each
    # launch uses; the events cost ~10 % of the step time, so they are kept out
    # of the timed region above
    trace = {k: {"launches": 0, "ms": 0.0, "busy_ms": 0.0, "flops": 0.0, "bytes": 0.0}
             for k in ("chol", "trsm", "gemm", "other")}
    traced_ms = None
    if not args.no_trace:
        for c in copies:
            c.copy_(P)
        torch.cuda.synchronize()
        fl.trace_enable(True)
        ev0.record(stream)
        for i in range(K):
            factor(copies[i], infos[i:i + 1])
        ev1.record(stream)
        torch.cuda.synchronize()
        traced_ms = ev0.elapsed_time(ev1) / K
        trace = fl.trace_collect()
        fl.trace_enable(False)

    # dominant kernel: the trailing update (SYRK/GEMM on FP64 matrix cores).
    # Its launches overlap each other (remainder and panel-row updates run on
    # two streams), so the rate is taken over their busy time per step: the
    # union of the launches' intervals, not the sum of their durations.
    g = trace["gemm"]
    busy_ms = g.get("busy_ms", 0.0)
    gemm_tflops = g["flops"] / (busy_ms * 1e-3) / 1e12 if busy_ms > 0 else 0.0
    per_launch_tflops = g["flops"] / (g["ms"] * 1e-3) / 1e12 if g["ms"] > 0 else 0.0
    roofline = {
        "kernel": "k_gemm_lds<F64> (trailing SYRK/GEMM, 128- and 64-tiles)",
        "bound": "mfma",
        "achieved": round(gemm_tflops, 3),
        "peak": PEAK_F64_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(gemm_tflops / PEAK_F64_TFLOPS, 4),
        "traffic": gemm_traffic(),
        "launches_per_step": g["launches"] / K,
        "gflop_per_step": round(g["flops"] / K / 1e9, 3),
        "busy_ms_per_step": round(busy_ms / K, 4),
        "summed_launch_ms_per_step": round(g["ms"] / K, 4),
        "per_launch_tflops": round(per_launch_tflops, 3),
        "avg_launch_ms": g["ms"] / max(1, g["launches"]),
        "avg_launch_gflop": g["flops"] / max(1, g["launches"]) / 1e9,
        "avg_launch_alg_bytes": g["bytes"] / max(1, g["launches"]),
        "measured_in": "instrumented pass of the same K steps (per-launch HIP events; achieved = trailing-update "
                       "flops / union of their launch intervals)",
        "instrumented_ms_per_step": None if traced_ms is None else round(traced_ms, 4),
    }
    breakdown = {k: {"launches": v["launches"] // K, "ms": round(v["ms"] / K, 4),
                     "busy_ms": round(v.get("busy_ms", 0.0) / K, 4),
                     "tflops": round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 3) if v["ms"] > 0 else None}
                 for k, v in trace.items() if k in ("chol", "trsm", "gemm", "other")}

    # ---- accuracy of the timed result (randomized backward-error estimate) --
    log("backward error of the FP64 factor")
    beta = factor_backward_error_est(P, copies[0])

    result = {
        "metric": METRIC,
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"dense SPD Cholesky n={n} FP64, A = B B^T + n I (B ~ N(0,1), PCG64 seed {args.seed})",
            "n": n, "nb": args.nb, "variant": {1: "bordered", 2: "left-looking", 3: "right-looking"}[args.variant],
            "lookahead": args.lookahead, "graph": bool(args.graph),
        },
        "pct_fp64_mfma_peak": round(100.0 * gflops / (PEAK_F64_TFLOPS * 1e3), 2),
        "beta_F": beta,
        "roofline": roofline,
        "kernels_per_step": breakdown,
    }
    del copies
    torch.cuda.empty_cache()

    if not args.no_mixed:
        result["mixed"] = mixed_leg(args, n, dev, fl, inputs, torch)
    if not args.no_batched:
        result["batched"] = batched_leg(args, dev, fl, inputs, torch)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_leg(P, n, args.cpu_seconds)
    if not args.no_extensions:
        # the conclusion's extensions of the loop at n = 8192 (see --extensions)
        recs = []
        ext = argparse.Namespace(**vars(args))
        ext.ext_ns, ext.ext_cases, ext.steps, ext.warmup, ext.no_cpu = "8192", "complex,lu,qr", 3, 1, True
        extensions_mode(ext, dev, fl, inputs, torch, emit=recs.append)
        result["extensions"] = {"n": 8192, "median_of": 3, "cases": recs}
    print(json.dumps(result), flush=True)
    return 0


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_gemm_lds_f64_n16384_traffic.md")


def gemm_traffic():
    """HBM bytes per trailing-update launch at this workload, from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary (calibrated against a
    plain copy); None when that summary is missing or was taken on other
    kernel sources."""
    from paper_1601_05871_amd import profile_summary

    try:
        with open(TRAFFIC_PROFILE) as f:
            text = f.read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            fields[k.strip("` ")] = v.strip("` ")
    if fields.get("source_hash") != profile_summary.gemm_source_hash():
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def factor_backward_error_est(A_dev, U_dev, k: int = 8, seed: int = 0) -> float:
    """||(A - U^T U) X||_F / (||A||_F ||X||_F) for X n x k N(0,1), formed on
    the host in FP64 numpy (A from its upper triangle)."""
    A = A_dev.cpu().numpy()
    U = np.triu(U_dev.cpu().numpy())
    n = A.shape[0]
    X = np.random.Generator(np.random.PCG64(seed)).standard_normal((n, k))
    Au = np.triu(A)
    AX = Au @ X + np.triu(A, 1).T @ X
    R = AX - U.T @ (U @ X)
    nA = np.sqrt(2.0 * np.sum(Au * Au) - np.sum(np.diag(A) ** 2))
    return float(np.linalg.norm(R) / (nA * np.linalg.norm(X)))


def mixed_leg(args, n, dev, fl, inputs, torch):
    """Time to solution of A0 X = B at backward error <= 1e-13 for every cell
    kappa x trail x nrhs: the FP64 path (flame_factor + one plain solve) against
    flame_solve_mixed (unit-diagonal scaling, the factorization with FP32 or
    BF16 trailing products, shifted retries after a breakdown, FP64
    refinement: IR, then preconditioned CG once IR stops halving eta), on the
    same A0 and B.  eta of every result is recomputed on the device in FP64."""
    kappas = [float(k) for k in args.kappas.split(",") if k]
    trails = [t for t in args.trails.split(",") if t]
    nrhs_list = [int(k) for k in args.nrhs.split(",") if k]
    tol = 1e-13
    W = torch.empty_strided((n, n), (1, n), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        rep = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), (time.perf_counter() - t0) * 1e3, rep

    def run_native(A0, b, x):
        W.copy_(A0)
        x.copy_(b)

        def go():
            info = fl.factor(W, variant=3, nb=args.nb, lookahead=args.lookahead)
            fl.solve(W, x)
            return info
        ms, wall, info = timed(go)
        return {"ms": round(ms, 3), "wall_ms": round(wall, 3), "info": int(info.item()),
                "eta": solve_backward_error_dev(A0, x, b, torch)}

    def run_mixed(A0, b, x, trail):
        x.copy_(b)
        ms, wall, rep = timed(lambda: fl.solve_mixed(A0, x, W=W, trail=trail, nb=0, tol=tol, max_iter=3000,
                                                     method="auto"))
        return {"ms": round(ms, 3), "wall_ms": round(wall, 3), "eta": solve_backward_error_dev(A0, x, b, torch),
                "eta_reported": rep["eta"], "iters": rep["iters"], "method": rep["method"],
                "shift": rep["shift"], "attempts": rep["attempts"], "status": rep["status"]}

    out = {"n": n, "tol": tol, "method": "auto (IR, then PCG)", "scaling": "unit diagonal",
           "cells": []}
    nmax = max(nrhs_list)
    for ki, kappa in enumerate(kappas):
        log(f"mixed leg: generating A0 = Q diag(s) Q^T, kappa={kappa:g}")
        A0 = inputs.spd_kappa_torch(n, kappa, args.seed, dev)
        Bh = inputs.rhs(n, nmax, args.seed)
        for nrhs in nrhs_list:
            b = torch.from_numpy(np.asfortranarray(Bh[:, :nrhs])).to(dev).as_strided((n, nrhs), (1, n))
            x = torch.empty_strided((n, nrhs), (1, n), dtype=torch.float64, device=dev)
            if ki == 0:  # warm-up of every path at this nrhs (workspace allocation, code loading)
                run_native(A0, b, x)
                for trail in trails:
                    run_mixed(A0, b, x, trail)
            log(f"mixed leg: kappa={kappa:g} nrhs={nrhs} native")
            base = run_native(A0, b, x)
            for trail in trails:
                log(f"mixed leg: kappa={kappa:g} nrhs={nrhs} {trail}")
                mix = run_mixed(A0, b, x, trail)
                ok = base["eta"] <= tol and mix["eta"] <= tol and mix["status"] == 0
                out["cells"].append({"kappa": kappa, "nrhs": nrhs, "trail": trail, "fp64": base, "mixed": mix,
                                     "speedup_vs_fp64": round(base["ms"] / mix["ms"], 3) if mix["ms"] > 0 else None,
                                     "equal_backward_error": bool(ok)})
            del b, x
        del A0
        torch.cuda.empty_cache()
    good = [c for c in out["cells"] if c["equal_backward_error"]]
    out["all_cells_converged"] = len(good) == len(out["cells"])
    if good:
        best = max(good, key=lambda c: c["speedup_vs_fp64"])
        out["best_speedup_vs_fp64"] = best["speedup_vs_fp64"]
        out["best_cell"] = {"kappa": best["kappa"], "nrhs": best["nrhs"], "trail": best["trail"]}
    del W
    torch.cuda.empty_cache()
    return out


def solve_backward_error_dev(A0, x, b, torch) -> float:
    """eta = ||b - A0 x||_inf / (||A0||_inf ||x||_inf + ||b||_inf) with torch
    FP64 on the device (measurement only; A0 symmetric from its upper part)."""
    Au = torch.triu(A0)
    S = Au + torch.triu(A0, 1).T
    r = b - S @ x
    nA = torch.max(torch.sum(torch.abs(S), dim=1))
    val = torch.max(torch.abs(r)) / (nA * torch.max(torch.abs(x)) + torch.max(torch.abs(b)))
    del S, Au
    return float(val.item())


def batched_leg(args, dev, fl, inputs, torch):
    """`args.batch` independent SPD matrices, n_i ~ U{16..512} (seeded, one
    B_i B_i^T + n_i I each), factored by one persistent launch replayed from a
    HIP graph; FP64 and FP32.  All matrices live in one buffer that is restored
    from a pristine copy between timed runs (outside the timed region)."""
    log(f"batched leg: generating {args.batch} matrices")
    sizes, mats = inputs.batch_torch(args.batch, args.seed, dev)
    offs = np.zeros(len(sizes) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes.astype(np.int64) ** 2)
    flops = float(sum(potrf_flops(int(n)) for n in sizes))
    out = {"count": int(args.batch), "n_range": [16, 512], "gflop_per_batch": round(flops / 1e9, 3)}
    for dt, code, name in ((torch.float64, fl.F64, "f64"), (torch.float32, fl.F32, "f32")):
        pristine = torch.empty(int(offs[-1]), dtype=dt, device=dev)
        for i, M in enumerate(mats):
            pristine[offs[i]:offs[i + 1]].copy_(M.T.reshape(-1))  # column-major bytes (M symmetric)
        work = torch.empty_like(pristine)
        esz = work.element_size()
        ns = torch.from_numpy(sizes).to(dev)
        ptrs = torch.from_numpy(work.data_ptr() + offs[:-1] * esz).to(dev)
        ldas = ns.clone()
        info = torch.zeros(len(sizes), dtype=torch.int32, device=dev)
        stream = torch.cuda.current_stream()
        times = []
        for it in range(max(1, args.warmup) + args.steps):
            work.copy_(pristine)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fl.batched_factor(ns, ptrs, ldas, info, dtype=code, graph=1)
            e1.record(stream)
            torch.cuda.synchronize()
            if it >= max(1, args.warmup):
                times.append(e0.elapsed_time(e1))
        bad = int(torch.count_nonzero(info).item())
        ms = float(np.median(times))
        out[name] = {"ms": round(ms, 4), "matrices_per_s": round(len(sizes) / (ms * 1e-3), 1),
                     "gflops": round(flops / (ms * 1e-3) / 1e9, 2), "nonzero_info": bad,
                     "frac_of_mfma_peak": round(flops / (ms * 1e-3) / 1e12 /
                                                (PEAK_F64_TFLOPS if name == "f64" else PEAK_F32_TFLOPS), 4)}
        log(f"batched {name}: {ms:.3f} ms, {out[name]['gflops']} GFLOP/s")
        del pristine, work
    del mats
    torch.cuda.empty_cache()
    return out


def table_mode(args, dev, fl, inputs, torch) -> int:
    """The single-matrix FP64 sweep: every n x nb x variant x seed cell, each
    factorization timed with HIP events on a resident copy (restored outside
    the timed region), median over seeds and repetitions; every block of the
    right-looking loop runs at the named nb (no smaller tail blocks)."""
    ns = [int(v) for v in args.table_ns.split(",") if v]
    nbs = [int(v) for v in args.table_nbs.split(",") if v]
    seeds = [int(v) for v in args.table_seeds.split(",") if v]
    reps = max(1, args.steps)
    names = {1: "bordered", 2: "left-looking", 3: "right-looking", 4: "by-blocks DAG"}
    stream = torch.cuda.current_stream()
    rows = []
    for n in ns:
        times = {(nb, v): [] for nb in nbs for v in (1, 2, 3)}
        for seed in seeds:
            log(f"table: n={n} seed={seed}")
            P = inputs.spd_bbt_torch(n, seed, dev)
            W = torch.empty_strided((n, n), (1, n), dtype=torch.float64, device=dev)
            info = torch.zeros(1, dtype=torch.int32, device=dev)
            for nb in nbs:
                for v in (1, 2, 3):
                    for r in range(1 + reps):
                        W.copy_(P)
                        torch.cuda.synchronize()
                        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        e0.record(stream)
                        fl.factor(W, variant=v, nb=nb, lookahead=args.lookahead, fixed_nb=True, info=info)
                        e1.record(stream)
                        torch.cuda.synchronize()
                        if int(info.item()) != 0:
                            log(f"breakdown n={n} nb={nb} variant={v}")
                            return 1
                        if r > 0:
                            times[(nb, v)].append(e0.elapsed_time(e1))
            # the by-blocks task DAG (its own 128-block grid, no nb)
            for r in range(1 + reps):
                W.copy_(P)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                fl.factor_by_blocks(W, info=info)
                e1.record(stream)
                torch.cuda.synchronize()
                if int(info.item()) != 0:
                    log(f"breakdown n={n} by-blocks")
                    return 1
                if r > 0:
                    times.setdefault((128, 4), []).append(e0.elapsed_time(e1))
            del P, W
            torch.cuda.empty_cache()
        for nb, v in [(nb, v) for nb in nbs for v in (1, 2, 3)] + [(128, 4)]:
            t = np.array(times[(nb, v)])
            med = float(np.median(t))
            tf = potrf_flops(n) / (med * 1e-3) / 1e12
            rec = {"n": n, "nb": nb, "variant": names[v], "ms_median": round(med, 3),
                   "ms_min": round(float(t.min()), 3), "ms_max": round(float(t.max()), 3),
                   "tflops": round(tf, 2), "pct_fp64_peak": round(100 * tf / PEAK_F64_TFLOPS, 1),
                   "samples": int(t.size)}
            rows.append(rec)
            print(json.dumps(rec), flush=True)
    print(f"\n| n | nb | variant | median ms | min ms | max ms | TFLOP/s | % FP64 peak |")
    print("|---|---|---|---|---|---|---|---|")
    for r in rows:
        print(f"| {r['n']} | {r['nb']} | {r['variant']} | {r['ms_median']} | {r['ms_min']} | {r['ms_max']} | "
              f"{r['tflops']} | {r['pct_fp64_peak']} |")
    return 0


def dag_mode(args, dev, fl, inputs, torch) -> int:
    """The by-blocks task DAG (one persistent launch over 128-blocks) against
    the default right-looking loop (nb = 512 schedule, lookahead 2) on the same
    seeded matrix: median of --steps factorizations after --warmup, each on a
    resident copy restored outside the timed region; the factor of each is
    checked against the other's (same U up to rounding)."""
    stream = torch.cuda.current_stream()
    for n in [int(v) for v in args.table_ns.split(",") if v]:
        P = inputs.spd_bbt_torch(n, 0, dev)
        W = torch.empty_strided((n, n), (1, n), dtype=torch.float64, device=dev)
        info = torch.zeros(1, dtype=torch.int32, device=dev)
        res, U = {}, {}
        for name, fn in (("loop", lambda: fl.factor(W, variant=fl.VAR_RIGHT, nb=512, lookahead=2, info=info)),
                         ("dag", lambda: fl.factor_by_blocks(W, info=info))):
            ts = []
            for r in range(args.warmup + args.steps):
                W.copy_(P)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                fn()
                e1.record(stream)
                torch.cuda.synchronize()
                if int(info.item()) != 0:
                    log(f"breakdown n={n} {name}")
                    return 1
                if r >= args.warmup:
                    ts.append(e0.elapsed_time(e1))
            res[name] = float(np.median(ts))
            U[name] = torch.triu(W).clone()
        rel = float((U["dag"] - U["loop"]).abs().max() / U["loop"].abs().max())
        rec = {"n": n, "loop_ms": round(res["loop"], 3), "dag_ms": round(res["dag"], 3),
               "dag_tflops": round(potrf_flops(n) / (res["dag"] * 1e-3) / 1e12, 2),
               "loop_tflops": round(potrf_flops(n) / (res["loop"] * 1e-3) / 1e12, 2),
               "dag_over_loop": round(res["dag"] / res["loop"], 3), "max_rel_diff_of_factors": rel}
        print(json.dumps(rec), flush=True)
        del P, W, U
        torch.cuda.empty_cache()
    return 0


def extensions_mode(args, dev, fl, inputs, torch, emit=None) -> int:
    """The loop's extensions the paper's conclusion lists: the complex
    Hermitian factorization A = U^H U (flame_factor on complex128, 4 n^3 / 3
    real flops) and the LU without pivoting (flame_lu, 2 n^3 / 3 flops), each
    the median of --steps runs after --warmup on a resident seeded matrix
    (B B^H + n I, complex Gaussian B; G + 2 (n + 1) I, Gaussian G) restored
    outside the timed region, with the backward error of the last run; beside
    them the oracle's unblocked loops (O8, O9, O10; one host thread) at
    --ext-oracle-n, one run each.  Householder QR (flame_qr, 4 n^3 / 3 flops
    for a square matrix) on a Gaussian matrix, checked by R^T R = A^T A, with
    the vendor geqrf through torch timed beside it.  One JSON line per case."""
    import time

    import oracle

    def out(rec):
        if emit is None:
            print(json.dumps(rec), flush=True)
        else:
            emit(rec)

    stream = torch.cuda.current_stream()

    def timed(P, fn, check):
        W = torch.empty_like(P)
        ts = []
        for r in range(args.warmup + args.steps):
            W.copy_(P)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            info = fn(W)
            e1.record(stream)
            torch.cuda.synchronize()
            if int(info.item()) != 0:
                raise RuntimeError("breakdown")
            if r >= args.warmup:
                ts.append(e0.elapsed_time(e1))
        return float(np.median(ts)), check(P, W)

    def herm_err(P, W):
        U = torch.triu(W)
        return float(torch.linalg.norm(P - U.conj().T @ U) / torch.linalg.norm(P))

    def lu_err(P, W):
        n = W.shape[0]
        L = torch.tril(W, -1) + torch.eye(n, dtype=W.dtype, device=W.device)
        return float(torch.linalg.norm(P - L @ torch.triu(W)) / torch.linalg.norm(P))

    def qr_err(P, W):  # R^T R = P^T P
        R = torch.triu(W)
        return float(torch.linalg.norm(P.T @ P - R.T @ R) / torch.linalg.norm(P) ** 2)

    cases = set(args.ext_cases.split(","))
    for n in [int(v) for v in args.ext_ns.split(",") if v]:
        g = torch.Generator(device=dev)
        g.manual_seed(args.seed)
        if "qr" in cases and not cases & {"complex", "lu"}:
            G = torch.randn(n, n, dtype=torch.float64, device=dev, generator=g)
            ms, err = timed(G.mT.contiguous().mT, lambda W: fl.qr(W)[1], qr_err)
            out({"case": "qr_householder", "n": n, "ms": round(ms, 3),
                 "tflops": round(4 * n ** 3 / 3 / (ms * 1e-3) / 1e12, 3), "gram_error": err})
            continue
        B = torch.randn(n, n, dtype=torch.complex128, device=dev, generator=g)
        P = B @ B.conj().T
        P.diagonal().copy_(P.diagonal().real + n)
        P = (torch.triu(P) + torch.triu(P, 1).conj().T).mT.contiguous().mT
        ms, err = timed(P, lambda W: fl.factor(W, variant=fl.VAR_RIGHT, nb=128), herm_err)
        out({"case": "complex_hermitian", "n": n, "ms": round(ms, 3),
             "tflops": round(4 * n ** 3 / 3 / (ms * 1e-3) / 1e12, 3), "backward_error": err})
        del B, P
        G = torch.randn(n, n, dtype=torch.float64, device=dev, generator=g)
        P = (G + 2.0 * (n + 1) * torch.eye(n, dtype=torch.float64, device=dev)).mT.contiguous().mT
        ms, err = timed(P, lambda W: fl.lu(W), lu_err)
        out({"case": "lu_nopiv", "n": n, "ms": round(ms, 3),
             "tflops": round(2 * n ** 3 / 3 / (ms * 1e-3) / 1e12, 3), "backward_error": err})
        del G, P
        G = torch.randn(n, n, dtype=torch.float64, device=dev, generator=g)
        P = G.mT.contiguous().mT
        ms, err = timed(P, lambda W: fl.qr(W)[1], qr_err)
        rec = {"case": "qr_householder", "n": n, "ms": round(ms, 3),
               "tflops": round(4 * n ** 3 / 3 / (ms * 1e-3) / 1e12, 3), "gram_error": err}
        try:  # the same factorization by the vendor library through torch (context)
            W = P.clone()
            torch.geqrf(W)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            torch.geqrf(W)
            e1.record(stream)
            torch.cuda.synchronize()
            rec["torch_geqrf_ms"] = round(e0.elapsed_time(e1), 3)
        except RuntimeError as e:
            rec["torch_geqrf_ms"] = None
            rec["torch_geqrf_error"] = str(e)[:120]
        out(rec)
        del G, P
        torch.cuda.empty_cache()
    if not args.no_cpu:
        n = args.ext_oracle_n
        A = inputs.hpd_bbh(n, args.seed)
        t0 = time.perf_counter()
        oracle.zpotrf(A)
        t_z = time.perf_counter() - t0
        A = inputs.diag_dominant(n, args.seed)
        t0 = time.perf_counter()
        oracle.getrf_nopiv(A)
        t_l = time.perf_counter() - t0
        A = inputs.qr_matrix(n, n, args.seed)
        t0 = time.perf_counter()
        oracle.geqrf(A)
        t_q = time.perf_counter() - t0
        out({"case": "oracle", "n": n, "cores": 1, "complex_hermitian_s": round(t_z, 3),
             "lu_nopiv_s": round(t_l, 3), "qr_householder_s": round(t_q, 3)})
    return 0


ICHOL_WORKLOADS = (((512, 512), 5, 0), ((512, 512), 5, 1), ((512, 512), 5, 2), ((64, 64, 64), 7, 0),
                   ((64, 64, 64), 7, 1), ((40, 40, 40), 27, 0), ((40, 40, 40), 27, 1))


def ichol_mode(args, dev, fl, inputs, torch) -> int:
    """Level(k) incomplete Cholesky of grid Laplacians (2-D 5-point 512^2 and
    3-D 7-point 64^3, about 5-7 entries per row, and 3-D 27-point 40^3, 27 per
    row, standing in for the paper's two classes of sparse matrices): the
    library's symbolic phase (host) with its own nested dissection, then the
    numeric phase on the device, median of --steps after --warmup (A's values
    resident on the device, the pool cleared and refilled inside each timed
    call); beside it the oracle's sequential incomplete factor (its own grid
    dissection and symbolic phase, untimed) on the host, one run; then the
    time to solution of A x = b by PCG with the factor (factor + iterations to
    ||r|| <= 1e-10 ||b||), beside the oracle's PCG on the smaller workloads.
    One JSON line per workload."""
    import time

    import oracle.ichol as oi

    stream = torch.cuda.current_stream()
    for dims, stencil, k in ICHOL_WORKLOADS:
        rp, ci, v = inputs.laplacian_grid(dims, stencil)
        n = len(rp) - 1
        t0 = time.perf_counter()
        P = fl.IcholPlan(n, rp, ci, k, leaf=256)
        t_an = time.perf_counter() - t0
        vals = torch.from_numpy(v).to(dev)
        info = torch.zeros(1, dtype=torch.int32, device=dev)
        ts = []
        for r in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            P.factor(vals, info=info)
            e1.record(stream)
            torch.cuda.synchronize()
            if int(info.item()) != 0:
                log(f"ichol breakdown {dims} k={k}: {int(info.item())}")
                return 1
            if r >= args.warmup:
                ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts))
        st = P.stats
        # the oracle, sequential C, on its own ordering of the same matrix
        order, _ = oi.nd_grid(dims, leaf=256)
        urp, uci, uv = oi.permute_upper(n, rp, ci, v, order)
        prp, pci, _ = oi.fill_pattern(n, urp, uci, k)
        ov = oi.values_on(prp, pci, urp, uci, uv)
        t0 = time.perf_counter()
        _, oinfo = oi.ichol(prp, pci, ov)
        cpu_ms = (time.perf_counter() - t0) * 1e3
        # PCG with the factor (time to solution of A x = b, b seeded, tol 1e-10)
        b = inputs.rhs(n, 1, 0)[:, 0]
        bd = torch.from_numpy(b).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.factor(vals, info=info)
        _, rep = P.pcg(vals, bd, tol=1e-10)
        pcg_ms = (time.perf_counter() - t0) * 1e3
        pcg_cpu = None
        if n * (k + 1) <= 300000:  # the oracle's PCG (scipy triangular solves) on the smaller workloads
            Uo, _ = oi.ichol(prp, pci, ov)
            t0 = time.perf_counter()
            _, oit, orel = oi.pcg(rp, ci, v, b, precond=lambda r: oi.triangular_apply(prp, pci, Uo, order, r),
                                  tol=1e-10)
            pcg_cpu = {"ms": round((time.perf_counter() - t0) * 1e3, 1), "iters": oit, "relres": orel}
        rec = {"workload": f"{len(dims)}-D {stencil}-point grid {'x'.join(map(str, dims))}", "n": n, "level": k,
               "nnz_a_upper": int((len(ci) + n) // 2), "nnz_u": st["nnz_u"], "blocks_per_side": st["nbt"],
               "blocks": st["nblocks"], "tasks": st["ntasks"], "gflop": round(st["flops"] / 1e9, 4),
               "analyze_host_ms": round(t_an * 1e3, 1), "factor_ms": round(ms, 3),
               "gflops": round(st["flops"] / (ms * 1e-3) / 1e9, 3),
               "oracle_cpu": {"ms": round(cpu_ms, 3), "nnz_u": int(len(pci)), "threads": 1, "info": oinfo},
               "gpu_over_cpu_speedup": round(cpu_ms / ms, 2),
               "pcg": {"factor_plus_solve_ms": round(pcg_ms, 2), "iters": rep["iters"], "relres": rep["relres"],
                       "status": rep["status"], "oracle_cpu": pcg_cpu}}
        print(json.dumps(rec), flush=True)
        P.close()
        del vals
        torch.cuda.empty_cache()
    return 0


def cpu_leg(P, n: int, seconds: float):
    """The CPU oracle (plain unblocked FP64 loop, OpenMP over columns) on the
    host cores, timed on the first J pivot steps of the same n x n matrix
    (J chosen for ~`seconds` of work); rate = the algorithmic flops of those
    steps / time."""
    import oracle

    log("cpu baseline: oracle on the host cores")
    A = np.asfortranarray(P.cpu().numpy())
    threads = oracle.max_threads()

    def step_flops(j0: int, j1: int) -> float:
        f = 0.0
        for j in range(j0, j1):
            r = n - j - 1
            f += 1 + r + r * (r + 1)  # sqrt, r divisions, r(r+1)/2 multiply-subtract pairs
        return f

    W = A.copy(order="F")
    t0 = time.perf_counter()
    oracle.potrf_inplace(W, n, n, threads=0, steps=2)
    t_probe = time.perf_counter() - t0
    J = int(max(2, min(n, 2 * seconds / max(t_probe, 1e-6))))
    W = A.copy(order="F")
    t0 = time.perf_counter()
    oracle.potrf_inplace(W, n, n, threads=0, steps=J)
    t = time.perf_counter() - t0
    fl = step_flops(0, J)
    return {"value": round(fl / t / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"first {J} of {n} pivot steps of the unblocked oracle on the same n={n} matrix "
                      f"({fl / 1e9:.1f} GFLOP, {t:.1f} s)"}


if __name__ == "__main__":
    sys.exit(main())
