"""LU without pivoting (flame_lu) against the oracle O9, element by element:
orders around the 64-blocks, padded leading dimensions, exact recovery inside
one block, breakdown, and a sampled n = 2048."""
import numpy as np
import pytest
import torch

import inputs
import oracle
import paper_1601_05871_amd as fl
from gpu_util import DEV, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,pad", [(1, 0), (2, 1), (33, 0), (64, 0), (65, 3), (127, 0), (128, 0), (129, 2),
                                   (300, 0), (700, 5)])
def test_lu_matches_oracle(n, pad):
    print(f"[lu] n={n} pad={pad}", flush=True)
    A = inputs.diag_dominant(n, 200 + n)
    Wo, io = oracle.getrf_nopiv(A)
    T = to_dev(A, n + pad)
    info = fl.lu(T)
    W = to_host(T)
    assert int(info.item()) == io == 0
    assert np.max(np.abs(np.triu(W) - np.triu(Wo))) <= 1e-13 * np.max(np.abs(np.triu(Wo)))
    assert np.max(np.abs(np.tril(W, -1) - np.tril(Wo, -1))) <= 1e-13
    assert oracle.lu_backward_error(A, W) <= 1e-14
    if pad:
        full = T.as_strided((n + pad, n), (1, n + pad)).cpu().numpy()
        assert np.all(np.isnan(full[n:]))  # padding rows never written


@pytest.mark.parametrize("n", [9, 64])
def test_lu_exact_inside_one_block(n):
    A, L, U = inputs.lu_exact(n, 5)
    T = to_dev(A)
    assert int(fl.lu(T).item()) == 0
    W = to_host(T)
    assert np.array_equal(np.triu(W), U)
    assert np.array_equal(np.tril(W, -1) + np.eye(n), L)


def test_lu_breakdown_column():
    n = 260
    A = inputs.diag_dominant(n, 9)
    A[150, 150] = np.nan
    _, io = oracle.getrf_nopiv(A)
    assert io == 151
    T = to_dev(A)
    assert int(fl.lu(T).item()) == io


def test_lu_sampled_large():
    n = 2048
    A = inputs.diag_dominant(n, 21)
    Wo, io = oracle.getrf_nopiv(A)
    T = to_dev(A)
    assert int(fl.lu(T).item()) == io == 0
    W = to_host(T)
    s = np.max(np.abs(np.triu(Wo)))
    for cols in (slice(0, 64), slice(n // 2, n // 2 + 64), slice(n - 64, n)):
        assert np.max(np.abs(W[:, cols] - Wo[:, cols])) <= 1e-13 * s
    assert oracle.lu_backward_error(A, W) <= 1e-14


def test_lu_lookahead_leading_block():
    """n = 4672: the lookahead is on (more than 2048 rows beyond the next
    step's) and the write-backs of A12 and A21 run on both streams (beyond
    4096 rows on the main one, below on the side one).  The leading 1024 x 1024
    block of the packed factors is the LU of A's leading block, against the
    oracle element by element; the whole factorization by its backward error."""
    n, k = 4672, 1024
    A = inputs.diag_dominant(n, 23)
    Wo, io = oracle.getrf_nopiv(np.asfortranarray(A[:k, :k]))
    T = to_dev(A)
    assert int(fl.lu(T).item()) == io == 0
    W = to_host(T)
    s = np.max(np.abs(np.triu(Wo)))
    assert np.max(np.abs(W[:k, :k] - Wo)) <= 1e-13 * s
    assert oracle.lu_backward_error(A, W) <= 1e-14
