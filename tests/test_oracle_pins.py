"""Pins of the CPU oracle against facts fixed by the paper and by mathematics,
not by the oracle itself (closed forms, exact-arithmetic inputs, an
independent library routine, high-precision brute force, the loop invariants of
the three derived variants, breakdown semantics).

The operation is A := Chol(A), A = U^T U with U upper (Fig. "dense-chol").
"""
import numpy as np
import pytest
import scipy.linalg as sl

import inputs
import oracle

U_EPS = np.finfo(np.float64).eps / 2  # unit roundoff u = 2^-53


# --- exact-arithmetic inputs -------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 7, 100, 513])
def test_minij_exact_and_lower_untouched(n):
    A = inputs.minij_scaled(n)
    W, info = oracle.potrf(A)
    assert info == 0
    assert np.array_equal(np.triu(W), inputs.minij_factor(n))
    # the strictly lower triangle is neither read nor written
    assert np.array_equal(np.tril(W, -1), np.tril(A, -1))


def test_minij_lower_garbage_is_ignored():
    n = 64
    A = inputs.minij_scaled(n)
    A[np.tril_indices(n, -1)] = np.nan  # poison: must not be read
    W, info = oracle.potrf(A)
    assert info == 0
    assert np.array_equal(np.triu(W), inputs.minij_factor(n))
    assert np.all(np.isnan(W[np.tril_indices(n, -1)]))


@pytest.mark.parametrize("n", [1, 5, 17, 29])
def test_pascal_exact(n):
    W, info = oracle.potrf(inputs.pascal(n))
    assert info == 0
    assert np.array_equal(np.triu(W), inputs.pascal_factor(n))


def test_diagonal_is_sqrt():
    d = np.random.Generator(np.random.PCG64(3)).uniform(0.1, 10.0, 37)
    W, info = oracle.potrf(np.asfortranarray(np.diag(d)))
    assert info == 0
    assert np.array_equal(np.diag(W), np.sqrt(d))
    assert np.array_equal(np.triu(W, 1), np.zeros((37, 37)))


def test_2x2_closed_form():
    # [[a, b], [b, c]] -> [[sqrt a, b / sqrt a], [0, sqrt(c - b^2 / a)]]
    A = np.asfortranarray([[4.0, 6.0], [6.0, 25.0]])
    W, info = oracle.potrf(A)
    assert info == 0
    assert np.array_equal(np.triu(W), np.array([[2.0, 3.0], [0.0, 4.0]]))


@pytest.mark.parametrize("n", [1, 2, 10, 200])
def test_laplacian_closed_form(n):
    # tridiag(-1, 2, -1): U_jj = sqrt((j+1)/j), U_{j,j+1} = -sqrt(j/(j+1)), 1-based j
    W, info = oracle.potrf(inputs.laplacian1d(n))
    assert info == 0
    j = np.arange(1, n + 1, dtype=np.float64)
    np.testing.assert_allclose(np.diag(W), np.sqrt((j + 1) / j), rtol=8 * U_EPS * 4, atol=0)
    if n > 1:
        np.testing.assert_allclose(np.diag(W, 1), -np.sqrt(j[:-1] / (j[:-1] + 1)), rtol=8 * U_EPS * 4, atol=0)
    assert not np.any(np.triu(W, 2))


# --- independent routines ----------------------------------------------------

@pytest.mark.parametrize("n,seed", [(1, 0), (50, 1), (300, 2), (777, 3)])
def test_against_lapack_potrf(n, seed):
    """LAPACK dpotrf (uplo = 'U') through scipy: the same definition computed
    by an independent routine; agreement to rounding."""
    A = inputs.spd_bbt(n, seed)
    W, info = oracle.potrf(A)
    assert info == 0
    U_lap = sl.cholesky(A, lower=False)
    # kappa(A) <~ 5: forward error ~ kappa * sqrt(n) * u, bounded by n * u
    assert oracle.forward_difference(W, U_lap) <= max(1, n) * U_EPS * 4
    assert oracle.factor_backward_error(A, W) <= 1e-14


@pytest.mark.parametrize("n,seed", [(3, 0), (8, 1), (12, 2)])
def test_against_mpmath_bruteforce(n, seed):
    """50-digit brute-force Cholesky (LDL^T, then square roots)."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    A = inputs.spd_bbt(n, seed)
    M = mp.matrix(A.tolist())
    L = mp.matrix(n, n)
    D = [mp.mpf(0)] * n
    for j in range(n):
        s = M[j, j] - sum(L[j, k] ** 2 * D[k] for k in range(j))
        D[j] = s
        L[j, j] = mp.mpf(1)
        for i in range(j + 1, n):
            L[i, j] = (M[i, j] - sum(L[i, k] * L[j, k] * D[k] for k in range(j))) / D[j]
    U_ex = np.zeros((n, n))
    for i in range(n):
        for j in range(i, n):
            U_ex[i, j] = float(L[j, i] * mp.sqrt(D[i]))
    W, info = oracle.potrf(A)
    assert info == 0
    err = np.max(np.abs(np.triu(W) - U_ex)) / np.max(np.abs(U_ex))
    assert err <= 4 * n * U_EPS


# --- breakdown ----------------------------------------------------------------

def test_breakdown_negative_pivot():
    A = np.asfortranarray(np.eye(9) * 4.0)
    A[5, 5] = -1.0
    _, info = oracle.potrf(A)
    assert info == 6


def test_breakdown_nan_pivot():
    A = inputs.spd_bbt(10, 0)
    A[3, 3] = np.nan
    _, info = oracle.potrf(A)
    assert info == 4


def test_breakdown_indefinite_minor():
    A = np.asfortranarray([[1.0, 2.0, 0.0], [2.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    W, info = oracle.potrf(A)
    assert info == 2
    assert W[0, 0] == 1.0 and W[0, 1] == 2.0  # column < info is final U


def test_zero_size():
    W, info = oracle.potrf(np.zeros((0, 0), order="F"))
    assert info == 0 and W.shape == (0, 0)


# --- blocked variants (O2) and the loop invariants -----------------------------

@pytest.mark.parametrize("b", [1, 3, 32, 64, 255, 256, 300])
@pytest.mark.parametrize("variant", [1, 2, 3])
def test_blocked_equals_unblocked_bitwise(b, variant):
    """Config 'n = 256, b = 32, seed 0' and neighbours: the blocked loop of
    Fig. "dense-chol" only regroups the unblocked arithmetic (b = 1), so with
    rank-1 terms applied in pivot order every variant is bit-identical."""
    A = inputs.spd_bbt(256, 0)
    W1, i1 = oracle.potrf(A)
    W2, i2 = oracle.potrf_blocked(A, b, variant)
    assert i1 == i2 == 0
    assert np.array_equal(np.triu(W2), np.triu(W1))
    assert np.array_equal(np.tril(W2, -1), np.tril(A, -1))


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_loop_invariants(variant):
    """After each iteration (A_TL is k x k) the matrix satisfies the variant's
    loop invariant, derived from the partitioned matrix expression
    U_TL = Chol(A_TL), U_TR = U_TL^{-T} A_TR, U_BR = Chol(A_BR - U_TR^T U_TR):
      var 1: A_TL = U_TL;                  A_TR, A_BR original
      var 2: A_TL = U_TL, A_TR = U_TR;     A_BR original
      var 3: A_TL = U_TL, A_TR = U_TR,     A_BR = A_BR - U_TR^T U_TR
    Checked bitwise against the final U and the b = 1 oracle after k steps, and
    the Schur complement also against a numpy product (to rounding)."""
    n, b = 100, 16
    A = inputs.spd_bbt(n, 5)
    U, _ = oracle.potrf(A)
    U = np.triu(U)
    it = 0
    for k in list(range(0, n, b))[1:] + [n]:
        it += 1
        W, info = oracle.potrf_blocked(A, b, variant, iters=it)
        assert info == 0
        TL = (slice(0, k), slice(0, k))
        TR = (slice(0, k), slice(k, n))
        BR = (slice(k, n), slice(k, n))
        assert np.array_equal(np.triu(W[TL]), U[TL])
        if variant == 1:
            assert np.array_equal(W[TR], A[TR])
            assert np.array_equal(np.triu(W[BR]), np.triu(A[BR]))
        elif variant == 2:
            assert np.array_equal(W[TR], U[TR])
            assert np.array_equal(np.triu(W[BR]), np.triu(A[BR]))
        else:
            assert np.array_equal(W[TR], U[TR])
            Wk, _ = oracle.potrf(A, steps=k)
            assert np.array_equal(np.triu(W[BR]), np.triu(Wk[BR]))
            S = A[BR] - U[TR].T @ U[TR]
            np.testing.assert_allclose(np.triu(W[BR]), np.triu(S), rtol=0,
                                       atol=64 * k * U_EPS * np.max(np.abs(A)))


def test_partial_steps_give_leading_rows():
    """O1 stopped after r steps already holds rows 0..r-1 of U (used to sample
    the factor of matrices too large for the whole oracle)."""
    A = inputs.spd_bbt(300, 9)
    U, _ = oracle.potrf(A)
    W, _ = oracle.potrf(A, steps=7)
    assert np.array_equal(np.triu(W[:7, :]), np.triu(U[:7, :]))


def test_literal_inverse_reading_fails():
    """The figure prints A12 := triu(A11)^{-1} A12.  Read literally, the
    blocked loop does not reconstruct A; the transposed solve does.  This pins
    the reading the oracle uses (numpy/scipy only)."""
    n, b = 64, 16
    A = inputs.spd_bbt(n, 11)

    def blocked(trans):
        W = np.array(A, order="F", copy=True)
        for k in range(0, n, b):
            e = min(k + b, n)
            W[k:e, k:e] = np.triu(sl.cholesky(np.triu(W[k:e, k:e]) + np.triu(W[k:e, k:e], 1).T, lower=False))
            W[k:e, e:] = sl.solve_triangular(np.triu(W[k:e, k:e]), W[k:e, e:], trans=trans, lower=False)
            W[e:, e:] -= W[k:e, e:].T @ W[k:e, e:]
        return np.triu(W)

    assert oracle.factor_backward_error(A, blocked("T")) < 1e-14
    assert oracle.factor_backward_error(A, blocked("N")) > 1e-3


# --- block operations ----------------------------------------------------------

def test_trsm_against_scipy():
    g = np.random.Generator(np.random.PCG64(7))
    U = np.triu(g.standard_normal((40, 40))) + 8 * np.eye(40)
    U = np.asfortranarray(U)
    U_lowgarbage = U + np.tril(g.standard_normal((40, 40)), -1)  # lower must be ignored
    X = np.asfortranarray(g.standard_normal((40, 23)))
    Y = oracle.trsm_upper_t(np.asfortranarray(U_lowgarbage), X)
    ref = sl.solve_triangular(U, X, trans="T", lower=False)
    np.testing.assert_allclose(Y, ref, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(U.T @ Y, X, rtol=1e-12, atol=1e-12)


def test_syrk_and_gemm_against_numpy():
    g = np.random.Generator(np.random.PCG64(8))
    P = np.asfortranarray(g.standard_normal((13, 29)))
    C = np.asfortranarray(g.standard_normal((29, 29)))
    D = oracle.syrk_upper(C, P)
    ref = C - P.T @ P
    np.testing.assert_allclose(np.triu(D), np.triu(ref), rtol=1e-13, atol=1e-13)
    assert np.array_equal(np.tril(D, -1), np.tril(C, -1))
    X = np.asfortranarray(g.standard_normal((13, 7)))
    E = oracle.gemm_tn(np.asfortranarray(C[:7, :]), X, P)
    np.testing.assert_allclose(E, C[:7, :] - X.T @ P, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("nrhs", [1, 5])
def test_solve_against_scipy(nrhs):
    A = inputs.spd_bbt(120, 4)
    U, _ = oracle.potrf(A)
    B = inputs.rhs(120, nrhs, 4)
    X = oracle.solve(np.triu(U), B)
    ref = sl.cho_solve((sl.cholesky(A, lower=False), False), B)
    np.testing.assert_allclose(X, ref.reshape(X.shape), rtol=1e-12, atol=1e-13)
    assert oracle.solve_backward_error(A, X, B) <= 1e-15


def test_solve_exact_minij():
    # A = minij: x = e_j-scaled exact check via A x = b with b = A 1
    n = 50
    A = inputs.minij_scaled(n)
    x = np.ones((n, 1))
    b = np.asfortranarray(A @ x)
    X = oracle.solve(inputs.minij_factor(n), b)
    np.testing.assert_allclose(X, x, rtol=0, atol=1e-9)


def test_backward_error_estimate_tracks_exact():
    A = inputs.spd_bbt(200, 1)
    U, _ = oracle.potrf(A)
    Up = np.triu(U).copy()
    Up[3, 7] *= 1 + 1e-9
    exact = oracle.factor_backward_error(A, Up)
    est = oracle.factor_backward_error_est(A, Up, seed=0, k=16)
    assert 0.05 * exact <= est <= 5 * exact


def test_flop_count():
    assert oracle.flops(1) == 1.0
    assert oracle.flops(3) == 9.0 + 4.5 + 0.5
