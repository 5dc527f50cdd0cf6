"""Selector inference kernel against the numpy MLP; the exhaustive autotuner."""
import numpy as np
import pytest
import torch

import inputs
import oracle
import paper_1601_05871_amd as fl
from paper_1601_05871_amd import selector as sel
from gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def test_logits_match_numpy_forward():
    p = sel.init_params(11)
    p["W3"] *= 10.0
    w = sel.flatten(p)
    fl.selector_load(w)
    try:
        g = np.random.Generator(np.random.PCG64(4))
        X = np.stack([sel.features(int(n), int(b), bool(d), float(k)) for n, b, d, k in
                      zip(np.exp(g.uniform(np.log(64), np.log(32768), 3000)).astype(int),
                          np.exp(g.uniform(0, np.log(10000), 3000)).astype(int), g.integers(0, 2, 3000),
                          10.0 ** g.uniform(0, 8, 3000))])
        zg = fl.select_logits(X)
        zo, _ = sel.forward(sel.unflatten(w), X.astype(np.float64))
        assert np.max(np.abs(zg - zo) / (1.0 + np.abs(zo))) <= 2e-5
        # select() is the argmax of the same logits (rows with a clear margin)
        for i in range(0, 3000, 97):
            s = np.sort(zo[i])
            if s[-1] - s[-2] < 1e-3:
                continue
            n = int(round(2.0 ** X[i, 0]))
            b = int(round(2.0 ** X[i, 1]))
            if sel.features(n, b, X[i, 2] == 1.0, 0.0)[:4].tolist() != X[i, :4].tolist() or X[i, 4] != 0.0:
                continue
            f64 = bool(X[i, 2])
            ok = [c for c in range(12) if sel.feasible(c, n, f64)]
            want = max(ok, key=lambda c: zo[i][c])
            if zo[i][want] - max(zo[i][c] for c in ok if c != want) < 1e-3:
                continue
            assert fl.select(n, b, fl.F64 if f64 else fl.F32)["cls"] == want
    finally:
        fl.selector_load(None)


def test_select_without_weights_is_unsupported():
    fl.selector_load(None)
    with pytest.raises(fl.FlameError) as e:
        fl.select(1000)
    assert e.value.status == fl.FLAME_ERR_UNSUPPORTED


def test_autotune_times_every_candidate_and_keeps_A():
    fl.selector_load(None)
    n = 300
    A = inputs.spd_bbt(n, 21)
    Ad = to_dev(A, ld=n + 5)
    t = fl.autotune(Ad, batch=50, reps=2)
    assert t.shape == (12,) and np.all(np.isfinite(t)) and np.all(t > 0)
    assert np.array_equal(to_host(Ad), A)
    # FP32 data: the mixed classes cannot run; above order 1024 the batched one
    t32 = fl.autotune(to_dev(A, dtype=torch.float32), batch=4, reps=1)
    assert np.all(np.isinf(t32[8:])) and np.all(np.isfinite(t32[:8]))
    big = inputs.spd_bbt(1100, 22)
    tb = fl.autotune(to_dev(big), batch=2, reps=1)
    assert np.isinf(tb[7]) and np.all(np.isfinite(tb[:7])) and np.all(np.isfinite(tb[8:]))
    # VAR_AUTO now takes the tuned candidate; the factor is still the oracle's
    Uo, _ = oracle.potrf(A, threads=8)
    info = fl.factor(Ad, variant=fl.VAR_AUTO, nb=0)
    assert int(info.item()) == 0
    Ug = to_host(Ad)
    assert np.max(np.abs(np.triu(Ug) - np.triu(Uo))) <= 1e-13 * np.max(np.abs(Uo))


def test_autotune_reports_failed_candidates_as_inf():
    n = 200
    A = inputs.spd_bbt(n, 3)
    A[10, 10] = -1.0
    t = fl.autotune(to_dev(A), reps=1)
    assert np.all(np.isinf(t[:8]))  # every factorization breaks down
    # the mixed classes cannot factor it either (a negative diagonal entry)
    assert np.all(np.isinf(t[8:]))
