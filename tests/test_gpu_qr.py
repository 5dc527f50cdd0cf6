"""Householder QR (flame_qr) against the oracle O10 element by element:
shapes around the 32-column panels and the 128-column blocks, tall matrices
whose panels span several workgroups (the exchange between them), padded
leading dimensions, zero columns and diagonal input (identity reflectors),
graded columns, and the full n = 8192 case (its first 64 columns against the
oracle, which needs only those columns, and all of R through the Gram identity
R^T R = A^T A).

Tolerances: Householder QR is backward stable, and on Gaussian inputs the
blocked and unblocked orders differ by a few hundred roundings at most in R
(relative to max |R|) and in the reflectors (|v| <= 1); 1e-12 is two orders
above what the blocked model of this loop shows at these sizes."""
import numpy as np
import pytest
import torch

import inputs
import oracle
import paper_1601_05871_amd as fl
from gpu_util import DEV, to_dev, to_host

pytestmark = pytest.mark.gpu


def _check_against_oracle(A, W, tau):
    m, n = A.shape
    Wo, to = oracle.geqrf(A)
    scale = max(1.0, float(np.max(np.abs(np.triu(Wo[:n])))))
    assert np.max(np.abs(np.triu(W[:n]) - np.triu(Wo[:n])), initial=0.0) <= 1e-12 * scale
    assert np.max(np.abs(np.tril(W, -1) - np.tril(Wo, -1)), initial=0.0) <= 1e-12
    assert np.max(np.abs(tau - to), initial=0.0) <= 1e-12
    if n:
        assert oracle.qr_backward_error(A, W, tau) <= 1e-14
        assert oracle.qr_orthogonality(W, tau) <= 1e-15 * m * 4


@pytest.mark.parametrize("m,n,pad", [(1, 1, 0), (2, 1, 0), (7, 5, 1), (32, 32, 0), (33, 33, 0), (64, 40, 0),
                                     (100, 100, 3), (129, 129, 0), (200, 131, 0), (300, 257, 0), (513, 200, 0),
                                     (1100, 300, 2), (1600, 1100, 0)])
def test_qr_matches_oracle(m, n, pad):
    print(f"[qr] m={m} n={n} pad={pad}", flush=True)
    A = inputs.qr_matrix(m, n, seed=m + 7 * n)
    T = to_dev(A, m + pad)
    tau, info = fl.qr(T)
    W = to_host(T)
    assert int(info.item()) == 0
    _check_against_oracle(A, W, tau.cpu().numpy())
    if pad:
        full = T.as_strided((m + pad, n), (1, m + pad)).cpu().numpy()
        assert np.all(np.isnan(full[m:]))  # padding rows never written


def test_qr_zero_columns_give_identity_reflectors():
    m, n = 700, 300
    A = inputs.qr_matrix(m, n, seed=4)
    A[:, 40] = 0.0
    A[:, 161] = 0.0
    T = to_dev(A)
    tau, info = fl.qr(T)
    W = to_host(T)
    t = tau.cpu().numpy()
    assert int(info.item()) == 0 and t[40] == 0.0 and t[161] == 0.0
    _check_against_oracle(A, W, t)


def test_qr_diagonal_input_is_exact():
    m, n = 600, 260  # every reflector is the identity: R = A bit for bit
    A = np.zeros((m, n), order="F")
    A[np.arange(n), np.arange(n)] = np.linspace(-3.0, 5.0, n)
    T = to_dev(A)
    tau, info = fl.qr(T)
    assert int(info.item()) == 0
    assert np.array_equal(to_host(T), A)
    assert np.array_equal(tau.cpu().numpy(), np.zeros(n))


def test_qr_graded_columns():
    m, n = 900, 400
    A = inputs.qr_matrix(m, n, seed=8, kappa=1e10)
    T = to_dev(A)
    tau, info = fl.qr(T)
    W = to_host(T)
    t = tau.cpu().numpy()
    assert int(info.item()) == 0
    assert oracle.qr_backward_error(A, W, t) <= 1e-14
    assert oracle.qr_orthogonality(W, t) <= 1e-15 * m * 4
    Wo, to = oracle.geqrf(A)
    # each row of R against the oracle's, relative to that row's size
    R, Ro = np.triu(W[:n]), np.triu(Wo[:n])
    rows = np.max(np.abs(Ro), axis=1)
    assert np.all(np.max(np.abs(R - Ro), axis=1) <= 1e-11 * rows)


def test_qr_tall_many_workgroups():
    # ceil(70000 / 512) = 137 workgroups exchange their sums for every column
    m, n = 70000, 40
    print(f"[qr] m={m} n={n}", flush=True)
    A = inputs.qr_matrix(m, n, seed=13)
    T = to_dev(A)
    tau, info = fl.qr(T)
    W = to_host(T)
    assert int(info.item()) == 0
    Wo, to = oracle.geqrf(A)
    scale = float(np.max(np.abs(np.triu(Wo[:n]))))
    assert np.max(np.abs(np.triu(W[:n]) - np.triu(Wo[:n]))) <= 1e-12 * scale
    assert np.max(np.abs(np.tril(W, -1) - np.tril(Wo, -1))) <= 1e-12
    assert np.max(np.abs(tau.cpu().numpy() - to)) <= 1e-12


def test_qr_wait_give_up_is_reported_and_recovers(monkeypatch):
    # the host makes every wait of the panel's exchange give up at once: info
    # is set, the later kernels skip, nothing waits; the next call is whole
    m, n = 1500, 64  # three workgroups exchange
    A = inputs.qr_matrix(m, n, seed=21)
    monkeypatch.setenv("FLAME_QR_SPIN_CAP", "-1")
    _, info = fl.qr(to_dev(A))
    assert int(info.item()) == 1
    monkeypatch.delenv("FLAME_QR_SPIN_CAP")
    T = to_dev(A)
    tau, info = fl.qr(T)
    assert int(info.item()) == 0
    _check_against_oracle(A, to_host(T), tau.cpu().numpy())


def test_qr_repeat_is_bitwise_identical():
    A = inputs.qr_matrix(1500, 700, seed=2)
    T1, T2 = to_dev(A), to_dev(A)
    t1, _ = fl.qr(T1)
    t2, _ = fl.qr(T2)
    assert torch.equal(T1, T2) and torch.equal(t1, t2)


def test_qr_no_columns():
    T = to_dev(np.ones((5, 0), order="F"))
    tau, info = fl.qr(T)
    assert int(info.item()) == 0


def test_qr_full_size_sampled():
    m = n = 8192
    print(f"[qr] full size m={m} n={n}", flush=True)
    A = inputs.qr_matrix(m, n, seed=11)
    T = to_dev(A)
    A_dev = T.clone()
    tau, info = fl.qr(T)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    # the first 64 columns of the factorization depend on A[:, :64] only
    k = 64
    Wo, to = oracle.geqrf(np.asfortranarray(A[:, :k]))
    W = T[:, :k].cpu().numpy()
    scale = float(np.max(np.abs(np.triu(Wo[:k]))))
    assert np.max(np.abs(np.triu(W[:k]) - np.triu(Wo[:k]))) <= 1e-12 * scale
    assert np.max(np.abs(np.tril(W, -1) - np.tril(Wo, -1))) <= 1e-12
    assert np.max(np.abs(tau[:k].cpu().numpy() - to)) <= 1e-12
    # all of R: R^T R = A^T A
    R = torch.triu(T)
    G = A_dev.T @ A_dev
    E = torch.linalg.norm(G - R.T @ R) / torch.linalg.norm(A_dev) ** 2
    assert float(E) <= 1e-13
    assert bool(torch.all(torch.isfinite(tau)))
