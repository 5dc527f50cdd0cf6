"""Cholesky-by-blocks without a GPU: the task list the library's persistent
kernel claims (counts, dependence order, and the per-iteration block
operations of the paper's example), and the oracle's by-blocks function
against what fixes it (the unblocked oracle, exact recovery of a factor
with the pattern, and the defining property of the block incomplete
factor)."""
import itertools

import numpy as np
import pytest

import inputs
import oracle
import paper_1601_05871_amd as fl

CHOL, TRSM, UPD = 0, 1, 2


def _example_pattern():
    """The 5 x 5 block structure of the paper's Cholesky-by-blocks example
    (Fig. example:cholesky-by-blocks): existing upper blocks 00, 04, 11, 13,
    14, 22, 23, 24, 33, 34, 44."""
    P = np.zeros((5, 5), dtype=np.uint8)
    for i, j in ((0, 0), (0, 4), (1, 1), (1, 3), (1, 4), (2, 2), (2, 3), (2, 4), (3, 3), (3, 4), (4, 4)):
        P[i, j] = 1
    return P


@pytest.mark.parametrize("nb", [1, 2, 3, 5, 8, 17])
def test_dense_task_counts(nb):
    """Dense block counts: N_b CHOL, N_b(N_b-1)/2 TRSM, N_b(N_b-1)/2 HERK
    (updates of diagonal blocks), N_b(N_b-1)(N_b-2)/6 GEMM; each task once."""
    t = fl.by_blocks_tasks(nb)
    assert len(set(t)) == len(t)
    chol = [x for x in t if x[0] == CHOL]
    trsm = [x for x in t if x[0] == TRSM]
    herk = [x for x in t if x[0] == UPD and x[2] == x[3]]
    gemm = [x for x in t if x[0] == UPD and x[2] < x[3]]
    assert len(chol) == nb
    assert len(trsm) == nb * (nb - 1) // 2
    assert len(herk) == nb * (nb - 1) // 2
    assert len(gemm) == nb * (nb - 1) * (nb - 2) // 6
    assert len(t) == len(chol) + len(trsm) + len(herk) + len(gemm)


def _check_order(t, exists):
    """Every task comes after every task it depends on (the property the
    kernel's progress argument rests on)."""
    pos = {x: q for q, x in enumerate(t)}
    for q, (ty, k, i, j) in enumerate(t):
        deps = []
        if ty == CHOL:
            deps += [(UPD, kk, k, k) for kk in range(k) if exists(kk, k)]
        elif ty == TRSM:
            deps += [(CHOL, k, k, k)] + [(UPD, kk, k, j) for kk in range(k) if exists(kk, k) and exists(kk, j)]
        else:
            deps += [(TRSM, k, k, i), (TRSM, k, k, j)]
            deps += [(UPD, kk, i, j) for kk in range(k) if exists(kk, i) and exists(kk, j)]
        for dd in deps:
            assert dd in pos, (dd, "missing")
            assert pos[dd] < q, ((ty, k, i, j), dd)


@pytest.mark.parametrize("nb", [1, 2, 6, 13])
def test_dense_dependence_order(nb):
    _check_order(fl.by_blocks_tasks(nb), lambda i, j: True)


def test_lookahead_in_the_order():
    """The diagonal block of iteration r + 1 is listed before the bulk of
    iteration r's updates (one iteration of lookahead)."""
    nb = 10
    t = fl.by_blocks_tasks(nb)
    pos = {x: q for q, x in enumerate(t)}
    for r in range(nb - 3):
        assert pos[(CHOL, r + 1, r + 1, r + 1)] < pos[(UPD, r, r + 3, r + 3)]


def test_paper_example_sequence():
    """The block operations per iteration for the example structure are those
    the paper lists (Fig. example:cholesky-by-blocks): CHOL of the diagonal
    block, TRSM of each existing block of the row, HERK / GEMM of each
    existing block the row's pairs reach."""
    P = _example_pattern()
    t = fl.by_blocks_tasks(5, P)
    per_iter = {k: sorted((ty, i, j) for ty, kk, i, j in t if kk == k) for k in range(5)}
    expect = {
        0: [(CHOL, 0, 0), (TRSM, 0, 4), (UPD, 4, 4)],
        1: [(CHOL, 1, 1), (TRSM, 1, 3), (TRSM, 1, 4), (UPD, 3, 3), (UPD, 3, 4), (UPD, 4, 4)],
        2: [(CHOL, 2, 2), (TRSM, 2, 3), (TRSM, 2, 4), (UPD, 3, 3), (UPD, 3, 4), (UPD, 4, 4)],
        3: [(CHOL, 3, 3), (TRSM, 3, 4), (UPD, 4, 4)],
        4: [(CHOL, 4, 4)],
    }
    assert per_iter == {k: sorted(v) for k, v in expect.items()}
    _check_order(t, lambda i, j: i == j or bool(P[i][j]))


def test_pattern_drops_missing_targets():
    """With a pattern that is not closed under fill, an update whose target
    block is missing is not generated."""
    P = np.eye(4, dtype=np.uint8)
    P[0, 1] = P[0, 3] = 1  # row 0 reaches (1, 3), which does not exist
    t = fl.by_blocks_tasks(4, P)
    assert (UPD, 0, 1, 3) not in t
    assert (UPD, 0, 1, 1) in t and (UPD, 0, 3, 3) in t
    _check_order(t, lambda i, j: i == j or bool(P[i][j]))


# ---- the oracle's by-blocks function ----------------------------------------

@pytest.mark.parametrize("n,b", [(1, 128), (100, 32), (300, 128), (333, 64)])
def test_oracle_by_blocks_dense_is_unblocked(n, b):
    """Dense pattern: the by-blocks loop takes the same rank-1 terms in pivot
    order as the unblocked oracle, so the factors agree bit for bit."""
    A = inputs.spd_bbt(n, 40)
    U1, i1 = oracle.potrf(A)
    U2, i2 = oracle.chol_by_blocks(A, None, b=b)
    assert i1 == i2 == 0
    assert np.array_equal(np.triu(U1), np.triu(U2))


def _pattern_factor(P, b, seed):
    """A U with the block pattern P (upper triangular blocks on the diagonal,
    positive diagonal), and A = U^T U."""
    nbt = P.shape[0]
    n = nbt * b
    g = np.random.Generator(np.random.PCG64(seed))
    U = np.zeros((n, n))
    for i, j in itertools.product(range(nbt), range(nbt)):
        if j >= i and (i == j or P[i][j]):
            blk = g.standard_normal((b, b))
            if i == j:
                blk = np.triu(blk) + np.diag(2.0 + np.abs(np.diag(blk)) + b ** 0.5)
            U[i * b:(i + 1) * b, j * b:(j + 1) * b] = blk
    U = np.triu(U)
    return np.asfortranarray(U), np.asfortranarray(U.T @ U)


def test_oracle_by_blocks_closed_pattern_recovers_factor():
    """The example structure is closed under fill: A = U^T U with U of that
    structure factors back to U (the unique factor), and blocks outside the
    pattern stay untouched (zero here)."""
    P = _example_pattern()
    U, A = _pattern_factor(P, 16, 5)
    W, info = oracle.chol_by_blocks(A, P.astype(bool), b=16)
    assert info == 0
    assert np.max(np.abs(np.triu(W) - U)) <= 1e-12 * np.max(np.abs(U))


def test_oracle_by_blocks_incomplete_property():
    """Fill dropped: the result U (zero outside the pattern) satisfies
    (U^T U)_ij = A_ij on every existing block, the defining property of the
    block incomplete Cholesky factor, while the dense factor of the same A
    differs."""
    b, nbt = 12, 5
    P = np.eye(nbt, dtype=bool)
    for i, j in ((0, 1), (0, 3), (1, 2), (2, 4), (0, 4)):
        P[i, j] = True
    n = nbt * b
    A = inputs.spd_bbt(n, 41)
    W, info = oracle.chol_by_blocks(A, P, b=b)
    assert info == 0
    U = np.zeros((n, n))
    for i, j in itertools.product(range(nbt), range(nbt)):
        if j >= i and P[i, j]:
            U[i * b:(i + 1) * b, j * b:(j + 1) * b] = W[i * b:(i + 1) * b, j * b:(j + 1) * b]
    U = np.triu(U)
    S = oracle.sym_from_upper(A)
    R = U.T @ U - S
    for i, j in itertools.product(range(nbt), range(nbt)):
        blk = R[i * b:(i + 1) * b, j * b:(j + 1) * b]
        if j >= i and P[i, j]:
            assert np.max(np.abs(blk)) <= 1e-12 * np.max(np.abs(S)), (i, j)
    Ud, _ = oracle.potrf(A)
    assert np.max(np.abs(np.triu(Ud) - U)) > 1e-3  # the dropped fill changes the factor


def test_oracle_by_blocks_breakdown():
    A = inputs.spd_bbt(200, 42)
    A[150, 150] = -1.0
    _, info = oracle.chol_by_blocks(A, None, b=64)
    assert info == 151
