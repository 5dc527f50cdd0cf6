"""Selector MLP (host side): parameter layout, the numpy forward pass against
a plain loop, the loss gradient against finite differences, and training on
a table with a known answer."""
import math

import numpy as np

import paper_1601_05871_amd as fl
from paper_1601_05871_amd import selector as sel


def test_param_layout_matches_header():
    assert sel.NPARAM == fl.SEL_NPARAM
    with open(__file__.replace("tests/test_selector_host.py", "include/flame.h")) as f:
        text = f.read()
    assert "#define FLAME_SEL_NPARAM (64 * 5 + 64 + 64 * 64 + 64 + 12 * 64 + 12)" in text
    p = sel.init_params(3)
    w = sel.flatten(p)
    assert w.dtype == np.float32 and w.size == sel.NPARAM
    q = sel.unflatten(w)
    for k in p:
        assert np.allclose(q[k], p[k].astype(np.float32))
    # W1 row-major first: w[j * 5 + k] = W1[j][k]
    assert w[7] == np.float32(p["W1"][1][2])


def test_class_table_matches_library():
    """The Python class names and feasibility rule agree with the library's
    class table (flame_select_class)."""
    for c, name in enumerate(sel.CLASS_NAMES):
        ch = fl.select_class(c)
        assert ch["cls"] == c
        assert ch["batched"] == (name == "batched")
        assert (ch["trail"] != "native") == name.startswith("mixed")
        if name.startswith("mixed"):
            assert ch["trail"] == name.split("-")[1] and ch["method"] == name.split("-")[2]
        elif name != "batched":
            variant = {"right": fl.VAR_RIGHT, "left": fl.VAR_LEFT, "bordered": fl.VAR_BORDERED}[name.split("-")[0]]
            assert ch["variant"] == variant and ch["nb"] == int(name.split("-")[1])
            assert ch["fixed_nb"] == name.endswith("fixed")
    assert sel.feasible(7, 1024, True) and not sel.feasible(7, 1025, True)
    assert sel.feasible(9, 100, True) and not sel.feasible(9, 100, False)


def test_forward_matches_plain_loops():
    p = sel.init_params(5)
    g = np.random.Generator(np.random.PCG64(0))
    X = g.uniform(0, 10, size=(4, 5))
    z, _ = sel.forward(p, X)
    for r in range(4):
        h1 = [max(0.0, p["b1"][j] + sum(p["W1"][j][k] * X[r][k] for k in range(5))) for j in range(64)]
        h2 = [max(0.0, p["b2"][j] + sum(p["W2"][j][k] * h1[k] for k in range(64))) for j in range(64)]
        out = [p["b3"][j] + sum(p["W3"][j][k] * h2[k] for k in range(64)) for j in range(12)]
        assert np.allclose(z[r], out, rtol=1e-12, atol=1e-12)


def test_gradient_matches_finite_differences():
    p = sel.init_params(1)
    g = np.random.Generator(np.random.PCG64(1))
    X = g.uniform(0, 4, size=(6, 5))
    S = 1.0 + g.uniform(0, 2, size=(6, 12))
    S[np.arange(6), g.integers(0, 12, 6)] = 1.0
    _, grad = sel.loss_and_grad(p, X, S)
    h = 1e-6
    for k, idx in (("W1", (3, 2)), ("b2", (7,)), ("W3", (5, 11)), ("W2", (10, 40))):
        p2 = {kk: v.copy() for kk, v in p.items()}
        p2[k][idx] += h
        lp, _ = sel.loss_and_grad(p2, X, S)
        p2[k][idx] -= 2 * h
        lm, _ = sel.loss_and_grad(p2, X, S)
        assert abs((lp - lm) / (2 * h) - grad[k][idx]) <= 1e-6 + 1e-4 * abs(grad[k][idx]), k


def _rule_times(n, batch, f64, kappa):
    """A known rule: batched for small orders in large batches, BF16 mixed for
    large well-conditioned FP64 systems, right-looking otherwise; infeasible
    classes +inf (as the autotuner reports them)."""
    t = np.full(12, 2.0)
    if n <= 1024 and batch >= 100:
        t[7] = 1.0
    elif f64 and n >= 4096 and kappa <= 1e3:
        t[9] = 1.0
    else:
        t[0] = 1.0
    for c in range(12):
        if not sel.feasible(c, n, f64):
            t[c] = np.inf
    return list(t)


def test_training_learns_a_known_rule():
    """The trained model reproduces a rule that depends on n, batch, dtype and
    kappa on shapes it has not seen."""
    import inputs

    recs = [{"n": n, "batch": b, "dtype": d, "kappa": k, "times_ms": _rule_times(n, b, d == "f64", k)}
            for n, b, d, k in inputs.selector_shapes(400, 1)]
    X, S = sel.rows(recs)
    p, hist = sel.train(X, S, epochs=3000, lr=3e-3)
    assert hist[-1][1] < hist[0][1]
    held = [{"n": n, "batch": b, "dtype": d, "kappa": k, "times_ms": _rule_times(n, b, d == "f64", k)}
            for n, b, d, k in ((300, 2000, "f64", 10.0), (8000, 1, "f64", 10.0), (8000, 1, "f64", 1e5),
                               (20000, 1, "f32", 10.0), (600, 1, "f64", 1e5))]
    res = sel.regret_table(p, held)
    assert res["mean_regret"] == 0.0, res
    assert set(res["chosen_classes"]) == {"batched", "mixed-bf16-auto", "right-512"}


def test_features():
    f = sel.features(1024, 1, True, 0.0)
    assert f.tolist() == [10.0, 0.0, 1.0, 0.0, 0.0]
    f = sel.features(64, 10000, False, 1e4)
    assert math.isclose(f[1], math.log2(10000), rel_tol=1e-6) and f[3] == 1.0 and math.isclose(f[4], 4.0)


def test_committed_weights_and_evaluation():
    """The committed selector weights have the library's layout and give
    finite logits; the committed held-out evaluation reports its regret."""
    import json
    import os

    with open(sel.DEFAULT_WEIGHTS) as f:
        w = np.array(json.load(f)["weights"], dtype=np.float32)
    assert w.size == fl.SEL_NPARAM
    z, _ = sel.forward(sel.unflatten(w), np.stack([sel.features(n, 1, d, 0.0) for n in (100, 5000) for d in (1, 0)]))
    assert np.all(np.isfinite(z))
    ev = os.path.join(os.path.dirname(sel.DEFAULT_WEIGHTS), "eval_heldout.json")
    with open(ev) as f:
        res = json.load(f)
    assert 0.0 <= res["mean_regret"] <= res["max_regret"]
    assert len(res["rows"]) >= 16
    # the committed evaluation: strictly better than every single fixed class,
    # and the choice depends on the shape
    assert res["mean_regret"] < res["best_fixed_mean_regret"]
    assert len(res["chosen_classes"]) >= 2
