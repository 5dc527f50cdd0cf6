"""Pins of O9, LU without pivoting by the loop of Fig. "dense-chol"'s pattern
(A = L U, L unit lower, U upper; the conclusion names LU among the
factorizations the pattern carries over to): exact recovery of integer
factors, the 2x2 closed form, LAPACK's partially pivoted LU through scipy on
column diagonally dominant matrices (where it does not pivot), the
reconstruction, breakdown on a zero pivot, and planted mistakes that each fail
a pin."""
import os

import numpy as np
import pytest
import scipy.linalg as sl

import inputs
import oracle
from oracle.build import SRC, build


def test_two_by_two_closed_form():
    # [[a, b], [c, d]] = [[1, 0], [c / a, 1]] [[a, b], [0, d - b c / a]]
    A = np.asfortranarray([[4.0, 3.0], [2.0, 5.0]])
    W, info = oracle.getrf_nopiv(A)
    assert info == 0
    assert np.array_equal(W, np.array([[4.0, 3.0], [0.5, 3.5]]))


@pytest.mark.parametrize("n,seed", [(1, 0), (7, 1), (40, 2), (90, 3)])
def test_exact_recovery(n, seed):
    A, L, U = inputs.lu_exact(n, seed)
    W, info = oracle.getrf_nopiv(A)
    assert info == 0
    assert np.array_equal(np.tril(W, -1) + np.eye(n), L)
    assert np.array_equal(np.triu(W), U)


@pytest.mark.parametrize("n", [10, 64, 129])
def test_against_scipy_lu(n):
    A = inputs.diag_dominant(n, n)
    P, L, U = sl.lu(A)
    assert np.array_equal(P, np.eye(n))  # no interchanges on this input
    W, info = oracle.getrf_nopiv(A)
    assert info == 0
    assert np.max(np.abs(np.tril(W, -1) - np.tril(L, -1))) <= 1e-13
    assert np.max(np.abs(np.triu(W) - U)) <= 1e-13 * np.max(np.abs(U))
    assert oracle.lu_backward_error(A, W) <= 1e-15


def test_zero_pivot_breakdown():
    A = np.asfortranarray([[1.0, 2.0, 3.0], [2.0, 4.0, 1.0], [1.0, 1.0, 1.0]])  # second pivot 4 - 2*2 = 0
    assert oracle.getrf_nopiv(A)[1] == 2
    B = inputs.diag_dominant(8, 1)
    B[0, 0] = np.nan
    assert oracle.getrf_nopiv(B)[1] == 1


MUTANTS = {
    "lu_update_sign": ("AT(A, lda, r, c) = AT(A, lda, r, c) - q;", "AT(A, lda, r, c) = AT(A, lda, r, c) + q;"),
    "lu_scales_row": ("for (int64_t r = j + 1; r < n; ++r) AT(A, lda, r, j) = AT(A, lda, r, j) / piv;",
                      "for (int64_t r = j + 1; r < n; ++r) AT(A, lda, j, r) = AT(A, lda, j, r) / piv;"),
    "lu_transposed_update": ("double q = AT(A, lda, r, j) * ujc;", "double q = AT(A, lda, j, r) * AT(A, lda, c, j);"),
    "lu_skips_last_row": ("            for (int64_t r = j + 1; r < n; ++r) {\n                double q",
                          "            for (int64_t r = j + 1; r < n - 1; ++r) {\n                double q"),
}


def _pins_pass(L) -> bool:
    saved = oracle._lib
    oracle._lib = L
    try:
        checks = []
        W, info = oracle.getrf_nopiv(np.asfortranarray([[4.0, 3.0], [2.0, 5.0]]))
        checks.append(info == 0 and np.array_equal(W, np.array([[4.0, 3.0], [0.5, 3.5]])))
        A, Le, Ue = inputs.lu_exact(40, 2)
        W, info = oracle.getrf_nopiv(A)
        checks.append(info == 0 and np.array_equal(np.triu(W), Ue) and
                      np.array_equal(np.tril(W, -1) + np.eye(40), Le))
        A = inputs.diag_dominant(64, 64)
        W, info = oracle.getrf_nopiv(A)
        checks.append(info == 0 and oracle.lu_backward_error(A, W) <= 1e-15)
        return all(checks)
    finally:
        oracle._lib = saved


def test_real_oracle_passes_lu_battery():
    assert _pins_pass(oracle.lib())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_lu_mutant_fails_a_pin(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    mpath = os.path.join(tmp_path, f"oracle_{name}.c")
    with open(mpath, "w") as f:
        f.write(src.replace(old, new))
    lpath = build(mpath, os.path.join(tmp_path, f"liboracle_{name}.so"))
    assert not _pins_pass(oracle.load(lpath))
