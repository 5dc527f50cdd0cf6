"""Cholesky-by-blocks on the device task DAG (flame_factor_by_blocks) against
the oracle: dense matrices of several orders (ragged last block, padded
leading dimension), exact structure, breakdown, determinism, and block
patterns (closed under fill, and with fill dropped) against the oracle's
by-blocks loop."""
import itertools

import numpy as np
import pytest
import torch

import inputs
import oracle
import paper_1601_05871_amd as fl
from gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

B = fl.BY_BLOCKS_TILE


def _rel(Ug, Uo):
    Ug, Uo = np.triu(Ug), np.triu(Uo)
    return float(np.max(np.abs(Ug - Uo)) / max(np.max(np.abs(Uo)), 1e-300))


@pytest.mark.parametrize("aligned", [True, False])
@pytest.mark.parametrize("n", [1, 5, 127, 128, 129, 300, 1000, 2600])
def test_by_blocks_dense_vs_oracle(n, aligned):
    """Both forms of the block update: operands staged through LDS (even
    leading dimension: 16-byte aligned columns) and read straight from
    memory (odd leading dimension)."""
    print(f"[by_blocks] dense n={n} aligned={aligned}", flush=True)
    A = inputs.spd_bbt(n, 50)
    Uo, io = oracle.potrf(A, threads=8)
    ld = n + 2 + (n & 1) if aligned else n + 3 - (n & 1)
    assert (ld % 2 == 0) == aligned
    Ad = to_dev(A, ld=ld)
    info = fl.factor_by_blocks(Ad)
    Ug = to_host(Ad)
    assert int(info.item()) == io == 0
    assert _rel(Ug, Uo) <= 1e-13
    assert oracle.factor_backward_error(A, Ug) <= 1e-14
    # the strictly lower triangle is never written
    assert np.array_equal(np.tril(Ug, -1), np.tril(to_host(to_dev(A, ld=ld)), -1))


def test_by_blocks_through_flame_factor_variant():
    n = 700
    A = inputs.spd_bbt(n, 51)
    Uo, _ = oracle.potrf(A, threads=8)
    Ad = to_dev(A)
    info = fl.factor(Ad, variant=fl.VAR_BY_BLOCKS, nb=0)
    assert int(info.item()) == 0
    assert _rel(to_host(Ad), Uo) <= 1e-13


def test_by_blocks_minij_exact():
    n = 1000
    A = inputs.minij_scaled(n)
    Ad = to_dev(A)
    assert int(fl.factor_by_blocks(Ad).item()) == 0
    assert np.array_equal(np.triu(to_host(Ad)), inputs.minij_factor(n))


@pytest.mark.parametrize("bad", [0, 77, 500, 999])
def test_by_blocks_breakdown(bad):
    """A clearly indefinite pivot stops the DAG (every workgroup exits) and
    is reported at its column."""
    A = inputs.spd_bbt(1000, 52)
    A[bad, bad] = -1.0
    Ad = to_dev(A)
    info = fl.factor_by_blocks(Ad)
    assert int(info.item()) == bad + 1
    # the next call starts clean
    A2 = inputs.spd_bbt(900, 53)
    Uo, _ = oracle.potrf(A2, threads=8)
    A2d = to_dev(A2)
    assert int(fl.factor_by_blocks(A2d).item()) == 0
    assert _rel(to_host(A2d), Uo) <= 1e-13


def test_by_blocks_deterministic():
    n = 1300
    A = inputs.spd_bbt(n, 54)
    outs = []
    for _ in range(2):
        Ad = to_dev(A)
        fl.factor_by_blocks(Ad)
        outs.append(to_host(Ad))
    assert np.array_equal(outs[0], outs[1])


def _example_pattern():
    P = np.zeros((5, 5), dtype=np.uint8)
    for i, j in ((0, 0), (0, 4), (1, 1), (1, 3), (1, 4), (2, 2), (2, 3), (2, 4), (3, 3), (3, 4), (4, 4)):
        P[i, j] = 1
    return P


def _pattern_factor(P, seed):
    nbt = P.shape[0]
    n = nbt * B
    g = np.random.Generator(np.random.PCG64(seed))
    U = np.zeros((n, n))
    for i, j in itertools.product(range(nbt), range(nbt)):
        if j >= i and (i == j or P[i][j]):
            blk = g.standard_normal((B, B))
            if i == j:
                blk = np.triu(blk) + np.diag(2.0 + np.abs(np.diag(blk)) + B ** 0.5)
            U[i * B:(i + 1) * B, j * B:(j + 1) * B] = blk
    U = np.triu(U)
    return np.asfortranarray(U), np.asfortranarray(U.T @ U)


def test_by_blocks_paper_example_pattern():
    """The example structure of the paper (closed under fill) with
    A = U^T U: the device factors back to U, matches the oracle's by-blocks
    loop, and leaves the blocks outside the pattern untouched."""
    P = _example_pattern()
    U, A = _pattern_factor(P, 6)
    A = np.asfortranarray(A)
    A[0:B, B:2 * B] = 7.0  # a block outside the pattern: must stay as it is
    Ad = to_dev(A, ld=A.shape[0] + 1)
    info = fl.factor_by_blocks(Ad, pattern=P)
    W = to_host(Ad)
    assert int(info.item()) == 0
    Wo, io = oracle.chol_by_blocks(A, P.astype(bool), b=B)
    assert io == 0
    assert np.all(W[0:B, B:2 * B] == 7.0)
    mask = np.kron(np.triu(P + np.eye(5, dtype=np.uint8)) > 0, np.ones((B, B), dtype=bool))
    assert np.max(np.abs(np.triu(W)[mask] - np.triu(Wo)[mask])) <= 1e-13 * np.max(np.abs(Wo))
    assert np.max(np.abs(np.triu(W)[mask] - U[mask])) <= 1e-12 * np.max(np.abs(U))


def test_by_blocks_incomplete_pattern_vs_oracle():
    """A pattern whose fill is dropped, on a ragged order: the device result
    equals the oracle's by-blocks loop on every existing block."""
    nbt = 7
    n = nbt * B - 37
    g = np.random.Generator(np.random.PCG64(8))
    P = np.triu(g.uniform(size=(nbt, nbt)) < 0.45).astype(np.uint8)
    np.fill_diagonal(P, 1)
    A = inputs.spd_bbt(n, 55)
    Ad = to_dev(A)
    info = fl.factor_by_blocks(Ad, pattern=P)
    W = to_host(Ad)
    Wo, io = oracle.chol_by_blocks(A, P.astype(bool), b=B)
    assert int(info.item()) == io == 0
    mask = np.kron(np.triu(P) > 0, np.ones((B, B), dtype=bool))[:n, :n]
    assert np.max(np.abs(np.triu(W)[mask] - np.triu(Wo)[mask])) <= 1e-13 * np.max(np.abs(Wo))
    # blocks outside the pattern are untouched
    assert np.array_equal(W[~mask & np.triu(np.ones((n, n), dtype=bool))], A[~mask & np.triu(np.ones((n, n), dtype=bool))])


def test_by_blocks_patterns_alternate():
    """The task lists of two patterns (and the dense one) alternate between
    calls: each call runs its own list."""
    P = _example_pattern()
    U, A = _pattern_factor(P, 9)
    D = inputs.spd_bbt(5 * B, 56)
    Do, _ = oracle.potrf(D, threads=8)
    for _ in range(2):
        Ad = to_dev(A)
        assert int(fl.factor_by_blocks(Ad, pattern=P).item()) == 0
        mask = np.kron(np.triu(P) > 0, np.ones((B, B), dtype=bool))
        assert np.max(np.abs(np.triu(to_host(Ad))[mask] - U[mask])) <= 1e-12 * np.max(np.abs(U))
        Dd = to_dev(D)
        assert int(fl.factor_by_blocks(Dd).item()) == 0
        assert _rel(to_host(Dd), Do) <= 1e-13
