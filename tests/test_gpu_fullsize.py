"""Full-size checks at n = 16384 in the benchmark's launch configuration
(right-looking, nb = 512, lookahead 2): an exact
input checked everywhere, a random input checked through properties that hold
at any size and on the rows the oracle can afford, and the mixed-precision
path with refinement."""
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


def test_fullsize_random_properties_and_leading_rows():
    J = 48  # rows of U the oracle computes (the first J pivot steps)
    P = inputs.spd_bbt_torch(N, 0, DEV)
    A = P.clone(memory_format=torch.preserve_format)
    assert A.stride(0) == 1
    info = _bench_factor(A)
    assert int(info.item()) == 0
    Uh = np.asfortranarray(A.cpu().numpy())
    Ph = np.asfortranarray(P.cpu().numpy())
    del A
    torch.cuda.empty_cache()
    # positive diagonal, finite entries
    diag = np.diag(Uh)
    assert np.all(diag > 0) and np.all(np.isfinite(np.triu(Uh)))
    # randomized backward error ||(A - U^T U) X||_F / (||A||_F ||X||_F), X n x 8
    U = np.triu(Uh)
    X = np.random.Generator(np.random.PCG64(0)).standard_normal((N, 8))
    Au = np.triu(Ph)
    AX = Au @ X + np.triu(Ph, 1).T @ X
    R = AX - U.T @ (U @ X)
    nA = np.sqrt(2.0 * np.sum(Au * Au) - np.sum(np.diag(Ph) ** 2))
    beta = float(np.linalg.norm(R) / (nA * np.linalg.norm(X)))
    assert beta <= 1e-14, beta
    del AX, R, Au, U
    # the first J rows of U against the oracle's first J pivot steps
    W = Ph.copy(order="F")
    assert oracle.potrf_inplace(W, N, N, threads=0, steps=J) == 0
    rows_o = np.triu(W[:J, :])
    rows_g = np.triu(Uh[:J, :])
    assert np.max(np.abs(rows_g - rows_o)) <= 1e-13 * np.max(np.abs(rows_o))


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
    # ||(A - U^T U) X||_F / (||A||_F ||X||_F), A from its upper triangle
    X = torch.randn(n, 8, dtype=torch.float64, device=DEV, generator=torch.Generator(device=DEV).manual_seed(0))
    Au = torch.triu(P)
    A = Au + torch.triu(P, 1).T.contiguous()
    R = A @ X - U.T.contiguous() @ (U @ X)
    beta = float(torch.linalg.norm(R) / (torch.linalg.norm(A) * torch.linalg.norm(X)))
    assert beta <= 1e-14, beta
