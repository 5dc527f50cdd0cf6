"""Pins of O8, the complex Hermitian factorization A = U^H U (the b = 1 loop
of Fig. "dense-chol" with the Hermitian update; complex data is one of the
extensions the conclusion lists).  None of the pins retypes the oracle's
formula: closed forms, exact recovery, the real special case (equal to O1 bit
for bit), numpy's complex Cholesky, the factorization's reconstruction, the
breakdown column against eigenvalues of leading blocks, and planted mistakes
that each fail a pin."""
import os

import numpy as np
import pytest

import inputs
import oracle
from oracle.build import SRC, build


def test_two_by_two_closed_form():
    # [[a, b], [conj b, c]] = U^H U with U = [[sqrt a, b / sqrt a], [0, sqrt(c - |b|^2 / a)]]
    A = np.array([[4.0, 2.0 + 2.0j], [2.0 - 2.0j, 11.0]])
    W, info = oracle.zpotrf(A)
    assert info == 0
    assert np.array_equal(np.triu(W), np.array([[2.0, 1.0 + 1.0j], [0.0, 3.0]]))
    assert W[1, 0] == 2.0 - 2.0j  # strictly lower triangle untouched


@pytest.mark.parametrize("n,seed", [(1, 0), (5, 1), (17, 2), (40, 3)])
def test_exact_recovery(n, seed):
    A, U = inputs.hpd_exact(n, seed)
    W, info = oracle.zpotrf(A)
    assert info == 0
    assert np.array_equal(np.triu(W), U)


def test_real_matrix_equals_real_oracle_bitwise():
    A = inputs.spd_bbt(50, 4)
    W, info = oracle.zpotrf(A.astype(np.complex128))
    Wr, ir = oracle.potrf(A)
    assert info == ir == 0
    assert np.array_equal(np.triu(W).real, np.triu(Wr))
    assert not np.any(np.triu(W).imag)


@pytest.mark.parametrize("n", [8, 33, 96])
def test_against_numpy_cholesky(n):
    A = inputs.hpd_bbh(n, n)
    W, info = oracle.zpotrf(A)
    assert info == 0
    U_np = np.linalg.cholesky(A).conj().T  # numpy: A = L L^H
    assert np.max(np.abs(np.triu(W) - U_np)) <= 1e-13 * np.max(np.abs(U_np))
    assert oracle.zfactor_backward_error(A, W) <= 1e-15
    assert np.all(np.diag(W).imag == 0) and np.all(np.diag(W).real > 0)


def test_breakdown_column_matches_leading_minors():
    A = inputs.hpd_bbh(30, 5)
    A[17, 17] = -40.0 * 30  # indefinite from column 18 on
    W, info = oracle.zpotrf(A)
    # first k whose leading k x k block is not positive definite
    first = next(k for k in range(1, 31) if np.linalg.eigvalsh(A[:k, :k]).min() <= 0)
    assert info == first
    B = inputs.hpd_bbh(6, 0)
    B[2, 2] = np.nan
    assert oracle.zpotrf(B)[1] == 3


MUTANTS = {
    "herk_no_conjugate": ("double pr = xr * yr + xi * yi;\n                double pi = xr * yi - xi * yr;",
                          "double pr = xr * yr - xi * yi;\n                double pi = xr * yi + xi * yr;"),
    "herk_imag_sign": ("double pi = xr * yi - xi * yr;", "double pi = xi * yr - xr * yi;"),
    "trsm_real_part_only": ("ZI(A, lda, j, c) = ZI(A, lda, j, c) / dr;", "ZI(A, lda, j, c) = ZI(A, lda, j, c);"),
    "herk_skips_diagonal": ("for (int64_t i = j + 1; i <= c; i++) {", "for (int64_t i = j + 1; i < c; i++) {"),
}


def _pins_pass(L) -> bool:
    saved = oracle._lib
    oracle._lib = L
    try:
        checks = []
        W, info = oracle.zpotrf(np.array([[4.0, 2.0 + 2.0j], [2.0 - 2.0j, 11.0]]))
        checks.append(info == 0 and np.array_equal(np.triu(W), np.array([[2.0, 1.0 + 1.0j], [0.0, 3.0]])))
        A, U = inputs.hpd_exact(17, 2)
        W, info = oracle.zpotrf(A)
        checks.append(info == 0 and np.array_equal(np.triu(W), U))
        A = inputs.hpd_bbh(33, 33)
        W, info = oracle.zpotrf(A)
        checks.append(info == 0 and oracle.zfactor_backward_error(A, W) <= 1e-15)
        return all(checks)
    finally:
        oracle._lib = saved


def test_real_oracle_passes_complex_battery():
    assert _pins_pass(oracle.lib())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_complex_mutant_fails_a_pin(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    mpath = os.path.join(tmp_path, f"oracle_{name}.c")
    with open(mpath, "w") as f:
        f.write(src.replace(old, new))
    lpath = build(mpath, os.path.join(tmp_path, f"liboracle_{name}.so"))
    assert not _pins_pass(oracle.load(lpath))
