"""Learned selector: timing sweep, training, evaluation.

The selector is a 3-layer FP32 MLP (features -> 64 -> 64 -> 12, ReLU) whose
inference runs in the library's HIP kernel (``flame_select``).  Its 12
classes are the library's distinct programs for solving SPD systems of one
order (``flame.h``: right-looking at 512 by position and at fixed 256 / 128 /
64, left-looking 128 / 256, bordered 256, the batched persistent kernel, and
the mixed-precision solve with FP32 or BF16 products refined by IR-then-CG or
by CG).  Features: log2 n, log2 batch, is_f64, is_f32, log10 kappa (0 when
unknown).  The batch size matters through the batched class (one launch for
the whole batch against one factorization per matrix), kappa through the
mixed classes (refinement steps grow with kappa u).

Pipeline (each step a subcommand):

  sweep  (GPU) the library's exhaustive autotuner (``flame_autotune``) times
         every class, per matrix, on seeded shapes (n, batch, dtype, kappa):
         n log-uniform in [64, 32768], batch in [1, 10000], FP64 with
         probability 3/4, kappa in [1, 1e6] (A = B B^T / n + sigma I, sigma
         setting kappa); writes the timing table.
  train  (CPU) fits the MLP to the table.  The loss is the expected slowdown
         sum_c softmax(z)_c t_c / t_best over the classes that can run
         (cost-sensitive, so near-ties cost little); full-batch Adam.
  eval   regret t(chosen) / t(best) - 1 on the held-out shapes, from the numpy
         forward pass and, with --device, from the HIP kernel; beside it the
         regret of the best single fixed class.

    python -m paper_1601_05871_amd.selector sweep --out sweep.json
    python -m paper_1601_05871_amd.selector train --sweep sweep.json --out weights.json
    python -m paper_1601_05871_amd.selector eval --sweep sweep.json --weights weights.json [--device]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

F, H, C = 5, 64, 12
NPARAM = H * F + H + H * H + H + C * H + C
HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "selector_data", "weights.json")

# class -> (name, runs FP32 data, largest order) as in flame.h
CLASS_NAMES = ("right-512", "right-256-fixed", "right-128-fixed", "right-64-fixed", "left-128", "left-256",
               "bordered-256", "batched", "mixed-f32-auto", "mixed-bf16-auto", "mixed-f32-cg", "mixed-bf16-cg")


def feasible(c: int, n: int, is_f64: bool) -> bool:
    """Whether class c can run a shape (the library's rule)."""
    if c == 7:
        return n <= 1024
    if c >= 8:
        return is_f64
    return True


def features(n: int, batch: int, is_f64: bool, kappa: float = 0.0) -> np.ndarray:
    return np.array([math.log2(max(n, 1)), math.log2(max(batch, 1)), 1.0 if is_f64 else 0.0,
                     0.0 if is_f64 else 1.0, math.log10(max(kappa, 1.0))], dtype=np.float32)


# ---- the MLP (numpy) ----------------------------------------------------------

def init_params(seed: int = 0) -> dict:
    g = np.random.Generator(np.random.PCG64(seed))

    def he(o, i):
        return g.standard_normal((o, i)) * math.sqrt(2.0 / i)

    return {"W1": he(H, F), "b1": np.zeros(H), "W2": he(H, H), "b2": np.zeros(H), "W3": he(C, H) * 0.1,
            "b3": np.zeros(C)}


def flatten(p: dict) -> np.ndarray:
    """Parameters in the library's order: W1[64][5], b1, W2[64][64], b2,
    W3[12][64], b3 (row-major, float32)."""
    return np.concatenate([p[k].reshape(-1) for k in ("W1", "b1", "W2", "b2", "W3", "b3")]).astype(np.float32)


def unflatten(w) -> dict:
    w = np.asarray(w, dtype=np.float64).reshape(-1)
    assert w.size == NPARAM
    out, o = {}, 0
    for k, shape in (("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (C, H)), ("b3", (C,))):
        size = int(np.prod(shape))
        out[k] = w[o:o + size].reshape(shape)
        o += size
    return out


def forward(p: dict, X: np.ndarray):
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    return h2 @ p["W3"].T + p["b3"], (X, z1, h1, z2, h2)


def _softmax(z):
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def loss_and_grad(p: dict, X, S, ce_weight: float = 0.1):
    """S: normalized times t_c / t_best (>= 1) per row.  Returns the mean
    expected slowdown + ce_weight * cross-entropy on argmin, and gradients."""
    z, (X0, z1, h1, z2, h2) = forward(p, X)
    P = _softmax(z)
    m = X.shape[0]
    exp_slow = np.sum(P * S, axis=1)
    best = np.argmin(S, axis=1)
    ce = -np.log(np.maximum(P[np.arange(m), best], 1e-300))
    loss = float(np.mean(exp_slow) + ce_weight * np.mean(ce))
    # d/dz of sum_c P_c S_c = P * (S - exp_slow); of CE = P - onehot
    onehot = np.zeros_like(P)
    onehot[np.arange(m), best] = 1.0
    dz = (P * (S - exp_slow[:, None]) + ce_weight * (P - onehot)) / m
    g = {"W3": dz.T @ h2, "b3": dz.sum(axis=0)}
    dh2 = dz @ p["W3"]
    dz2 = dh2 * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (z1 > 0)
    g["W1"] = dz1.T @ X0
    g["b1"] = dz1.sum(axis=0)
    return loss, g


def train(X, S, epochs: int = 4000, lr: float = 3e-3, seed: int = 0, ce_weight: float = 0.1):
    p = init_params(seed)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    b1, b2, eps = 0.9, 0.999, 1e-8
    hist = []
    for t in range(1, epochs + 1):
        loss, g = loss_and_grad(p, X, S, ce_weight)
        for k in p:
            m[k] = b1 * m[k] + (1 - b1) * g[k]
            v[k] = b2 * v[k] + (1 - b2) * g[k] ** 2
            p[k] = p[k] - lr * (m[k] / (1 - b1 ** t)) / (np.sqrt(v[k] / (1 - b2 ** t)) + eps)
        if t % 500 == 0 or t == 1:
            hist.append((t, loss))
    return p, hist


# ---- data -----------------------------------------------------------------------

def normalized(times) -> np.ndarray:
    """t_c / t_best; classes that cannot run or failed get 10x the slowest."""
    t = np.array(times, dtype=np.float64)
    finite = np.isfinite(t)
    worst = np.max(t[finite]) if finite.any() else 1.0
    t[~finite] = 10.0 * worst
    return t / np.min(t)


def rows(records):
    X = np.array([features(r["n"], r["batch"], r["dtype"] == "f64", r["kappa"]) for r in records], dtype=np.float64)
    S = np.array([normalized(r["times_ms"]) for r in records])
    return X, S


def choose(p: dict, r: dict) -> int:
    """The selector's class for a record: argmax of the logits over the
    classes that can run it (as flame_select)."""
    z, _ = forward(p, features(r["n"], r["batch"], r["dtype"] == "f64", r["kappa"])[None, :])
    ok = [c for c in range(C) if feasible(c, r["n"], r["dtype"] == "f64")]
    return max(ok, key=lambda c: z[0][c])


def regret_table(p: dict, records) -> dict:
    out_rows = []
    for r in records:
        c = choose(p, r)
        s = normalized(r["times_ms"])
        out_rows.append({"n": r["n"], "batch": r["batch"], "dtype": r["dtype"], "kappa": r["kappa"],
                         "chosen": CLASS_NAMES[c], "best": CLASS_NAMES[int(np.argmin(s))],
                         "regret": float(s[c] - 1.0)})
    reg = np.array([x["regret"] for x in out_rows])
    # baseline: the single fixed class with the lowest mean regret on these shapes
    S = np.array([normalized(r["times_ms"]) for r in records]) - 1.0
    fixed = int(np.argmin(S.mean(axis=0)))
    return {"mean_regret": float(reg.mean()), "median_regret": float(np.median(reg)),
            "p95_regret": float(np.percentile(reg, 95)), "max_regret": float(reg.max()),
            "exact_best_fraction": float(np.mean(reg == 0.0)),
            "chosen_classes": sorted({x["chosen"] for x in out_rows}),
            "best_fixed_choice": CLASS_NAMES[fixed], "best_fixed_mean_regret": float(S[:, fixed].mean()),
            "best_fixed_max_regret": float(S[:, fixed].max()), "rows": out_rows}


# ---- commands ---------------------------------------------------------------------

def cmd_sweep(args) -> int:
    import torch

    sys.path.insert(0, os.path.dirname(HERE))
    import inputs
    import paper_1601_05871_amd as fl

    fl.lib()
    dev = torch.device("cuda:0")
    sets = {"train": inputs.selector_shapes(args.count, args.seed),
            "heldout": inputs.selector_shapes(args.heldout, args.seed + 1)}
    out = {"command": " ".join(sys.argv), "classes": list(CLASS_NAMES), "records": []}
    for split, shapes in sets.items():
        for k, (n, batch, dt, kappa) in enumerate(shapes):
            t0 = time.time()
            A = inputs.spd_wishart_shift_torch(n, kappa, 7000 + k, dev,
                                               dtype=torch.float64 if dt == "f64" else torch.float32)
            reps = 3 if n <= 4096 else (2 if n <= 16384 else 1)
            t = fl.autotune(A, batch=batch, reps=reps)
            del A
            torch.cuda.empty_cache()
            rec = {"split": split, "n": n, "batch": batch, "dtype": dt, "kappa": kappa, "reps": reps,
                   "times_ms": [None if not np.isfinite(x) else round(float(x), 5) for x in t]}
            out["records"].append(rec)
            b = int(np.argmin(t))
            print(f"[sweep] {split} n={n} batch={batch} {dt} kappa={kappa:.3g}: best {CLASS_NAMES[b]} "
                  f"{t[b]:.4f} ms/matrix ({time.time() - t0:.1f} s)", flush=True)
            with open(args.out, "w") as f:
                json.dump(out, f, indent=1)
    return 0


def _load_records(path, split):
    with open(path) as f:
        data = json.load(f)
    recs = []
    for r in data["records"]:
        if r["split"] == split:
            r = dict(r)
            r["times_ms"] = [np.inf if x is None else x for x in r["times_ms"]]
            recs.append(r)
    return recs


def cmd_train(args) -> int:
    recs = _load_records(args.sweep, "train")
    X, S = rows(recs)
    p, hist = train(X, S, epochs=args.epochs, lr=args.lr, seed=args.seed, ce_weight=args.ce_weight)
    w = flatten(p)
    res = regret_table(p, recs)
    with open(args.out, "w") as f:
        json.dump({"nparam": NPARAM, "weights": [float(x) for x in w], "train_loss": hist,
                   "train_mean_regret": res["mean_regret"], "sweep": os.path.basename(args.sweep),
                   "command": " ".join(sys.argv)}, f)
    print(f"trained on {len(recs)} timed shapes; final loss {hist[-1][1]:.4f}; "
          f"train mean regret {res['mean_regret']:.4f}")
    return 0


def cmd_eval(args) -> int:
    with open(args.weights) as f:
        w = np.array(json.load(f)["weights"], dtype=np.float32)
    p = unflatten(w)
    recs = _load_records(args.sweep, "heldout")
    res = regret_table(p, recs)
    if args.device:
        sys.path.insert(0, os.path.dirname(HERE))
        import paper_1601_05871_amd as fl

        fl.selector_load(w)
        agree = 0
        for row, r in zip(res["rows"], recs):
            ch = fl.select(r["n"], r["batch"], fl.F64 if r["dtype"] == "f64" else fl.F32, r["kappa"])
            agree += int(CLASS_NAMES[ch["cls"]] == row["chosen"])
        res["device_agrees"] = f"{agree}/{len(recs)}"
    res["command"] = " ".join(sys.argv)
    text = json.dumps(res, indent=1)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(f"held-out: {len(recs)} shapes, mean regret {res['mean_regret']:.4f}, max {res['max_regret']:.4f}, "
          f"best chosen {res['exact_best_fraction']:.2f}, classes chosen {res['chosen_classes']}; best fixed "
          f"{res['best_fixed_choice']}: mean {res['best_fixed_mean_regret']:.4f}, max "
          f"{res['best_fixed_max_regret']:.4f}" + (f", device agrees {res['device_agrees']}" if args.device else ""))
    return 0


def load_default(path: str = DEFAULT_WEIGHTS) -> None:
    """Loads the committed trained weights into the library."""
    import paper_1601_05871_amd as fl

    with open(path) as f:
        fl.selector_load(np.array(json.load(f)["weights"], dtype=np.float32))


def main() -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("sweep")
    a.add_argument("--out", required=True)
    a.add_argument("--count", type=int, default=64)
    a.add_argument("--heldout", type=int, default=24)
    a.add_argument("--seed", type=int, default=9000)
    b = sub.add_parser("train")
    b.add_argument("--sweep", required=True)
    b.add_argument("--out", required=True)
    b.add_argument("--epochs", type=int, default=12000)
    b.add_argument("--lr", type=float, default=1e-3)
    b.add_argument("--seed", type=int, default=0)
    b.add_argument("--ce-weight", type=float, default=0.05)
    c = sub.add_parser("eval")
    c.add_argument("--sweep", required=True)
    c.add_argument("--weights", required=True)
    c.add_argument("--out")
    c.add_argument("--device", action="store_true")
    args = ap.parse_args()
    return {"sweep": cmd_sweep, "train": cmd_train, "eval": cmd_eval}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())
