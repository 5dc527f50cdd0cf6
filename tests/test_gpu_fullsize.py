"""Full-size checks at n = 16384 in the benchmark's launch configuration
(right-looking, nb = 512, lookahead 2): an exact input checked everywhere, a
random input checked element by element against the whole oracle factor
(about 40 s of the oracle on 16 host cores) and through the randomized
backward error, the n = 10240 early-remainder schedule (eager and graph)
against the whole oracle factor, and the mixed-precision solve."""
import time

import numpy as np
import pytest
import torch

import inputs
import oracle
import paper_1601_05871_amd as fl

pytestmark = pytest.mark.gpu

N = 16384
DEV = "cuda:0"


def _bench_factor(A, trail="native"):
    return fl.factor(A, variant=fl.VAR_RIGHT, nb=512, lookahead=2, trail=trail)


def _minij_device(n):
    """Scaled min(i, j) (exact factor U_ij = d_j) built on the device."""
    d = torch.pow(2.0, (torch.arange(n, device=DEV) % 7 - 3).to(torch.float64))
    idx = torch.arange(1, n + 1, device=DEV, dtype=torch.float64)
    A = torch.minimum(idx[:, None], idx[None, :])
    A.mul_(d[:, None]).mul_(d[None, :])
    return A, d  # symmetric: row-major bytes = column-major bytes


def test_fullsize_exact_minij():
    A, d = _minij_device(N)
    info = _bench_factor(A.T)  # column-major view of the same bytes
    assert int(info.item()) == 0
    U = torch.triu(A.T)
    expect = torch.triu(d[None, :].expand(N, N))
    assert torch.equal(U, expect)


def _oracle_full(P_host, n):
    """The oracle's whole factor (OpenMP over columns, bitwise the serial one)."""
    W = P_host.copy(order="F")
    t0 = time.time()
    print(f"[fullsize] oracle factor n={n} on {oracle.max_threads()} threads", flush=True)
    assert oracle.potrf_inplace(W, n, n, threads=0) == 0
    print(f"[fullsize] oracle done in {time.time() - t0:.1f} s", flush=True)
    return W


def _rand_beta(P_host, U):
    """||(A - U^T U) X||_F / (||A||_F ||X||_F), X n x 8 Gaussian, A from its
    upper triangle (the randomized estimate of the factor backward error)."""
    n = U.shape[0]
    X = np.random.Generator(np.random.PCG64(0)).standard_normal((n, 8))
    Au = np.triu(P_host)
    AX = Au @ X + np.triu(P_host, 1).T @ X
    R = AX - U.T @ (U @ X)
    nA = np.sqrt(2.0 * np.sum(Au * Au) - np.sum(np.diag(P_host) ** 2))
    return float(np.linalg.norm(R) / (nA * np.linalg.norm(X)))


def test_fullsize_random_vs_whole_oracle():
    P = inputs.spd_bbt_torch(N, 0, DEV)
    A = P.clone(memory_format=torch.preserve_format)
    assert A.stride(0) == 1
    info = _bench_factor(A)
    assert int(info.item()) == 0
    Uh = np.asfortranarray(A.cpu().numpy())
    Ph = np.asfortranarray(P.cpu().numpy())
    del A, P
    torch.cuda.empty_cache()
    U = np.triu(Uh)
    del Uh
    assert np.all(np.diag(U) > 0) and np.all(np.isfinite(U))
    beta = _rand_beta(Ph, U)
    assert beta <= 1e-14, beta
    Uo = np.triu(_oracle_full(Ph, N))
    # every upper element: max |U_gpu - U_oracle| / max |U_oracle| <= 1e-13
    err = float(np.max(np.abs(U - Uo)) / np.max(np.abs(Uo)))
    assert err <= 1e-13, err


def test_fullsize_mixed_refinement():
    kappa = 1e4
    A0 = inputs.spd_kappa_torch(N, kappa, 0, DEV)
    b = torch.from_numpy(inputs.rhs(N, 1, 0)).to(DEV).as_strided((N, 1), (1, N))
    W = A0.clone(memory_format=torch.preserve_format)
    x = b.clone()
    info = _bench_factor(W, trail="f32")
    assert int(info.item()) == 0
    rep = fl.solve(W, x, A0=A0, tol=1e-13, max_iter=30)
    assert rep["status"] == fl.FLAME_OK and rep["eta"] <= 1e-13, rep
    # eta recomputed independently in FP64 on the host
    Ah = np.asfortranarray(A0.cpu().numpy())
    xh = x.cpu().numpy()
    bh = b.cpu().numpy()
    assert oracle.solve_backward_error(Ah, xh, bh) <= 1e-13


def test_graph_replays_match_eager_with_early_remainder():
    """n = 10240, nb = 512: the remainder update is launched ahead of the
    panel-row update (more than 8192 rows below the next panel) on a second
    stream; the captured graph, replayed twice, gives the eager factor bit for
    bit, and the factor's randomized backward error is at FP64 level."""
    n = 10240
    P = inputs.spd_bbt_torch(n, 3, DEV)
    U_eager = P.clone(memory_format=torch.preserve_format)
    info = fl.factor(U_eager, variant=fl.VAR_RIGHT, nb=512, lookahead=2)
    assert int(info.item()) == 0
    s = torch.cuda.Stream()
    outs = []
    with torch.cuda.stream(s):
        for _ in range(2):
            W = P.clone(memory_format=torch.preserve_format)
            info = fl.factor(W, variant=fl.VAR_RIGHT, nb=512, lookahead=2, graph=1)
            s.synchronize()
            assert int(info.item()) == 0
            outs.append(torch.triu(W))
            del W
    U = torch.triu(U_eager)
    assert torch.equal(outs[0], U) and torch.equal(outs[1], U)
    del outs, U_eager
    Uh = U.cpu().numpy()
    Ph = np.asfortranarray(P.cpu().numpy())
    del U, P
    torch.cuda.empty_cache()
    Uh = np.asfortranarray(Uh)
    assert _rand_beta(Ph, Uh) <= 1e-14
    # every upper element against the whole oracle factor
    Uo = np.triu(_oracle_full(Ph, n))
    err = float(np.max(np.abs(Uh - Uo)) / np.max(np.abs(Uo)))
    assert err <= 1e-13, err
