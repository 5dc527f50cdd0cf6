"""Mutation check of the oracle's pins: plausible mistakes (a dropped term, a
wrong sign, an off-by-one bound, a transposed operand, the literal reading of
the garbled TRSM, a weakened breakdown test) are planted in copies of the
oracle source, compiled on the CPU, and each must fail at least one pin.
The real oracle is never modified."""
import os

import numpy as np
import pytest
import scipy.linalg as sl

import inputs
import oracle
from oracle.build import SRC, build

MUTANTS = {
    "no_sqrt": ("double d = sqrt(a);", "double d = a;"),
    "update_sign": ("col[i] = col[i] - p;", "col[i] = col[i] + p;"),
    "update_skips_diagonal": ("for (int64_t i = j + 1; i <= c; ++i) {", "for (int64_t i = j + 1; i < c; ++i) {"),
    "update_wrong_row": ("double p = row[i] * ujc;", "double p = row[c] * ujc;"),
    "trsm_untransposed": ("double p = AT(U, ldu, s, r) * x[s];\n                x[r] = x[r] - p;",
                          "double p = AT(U, ldu, r, s) * x[s];\n                x[r] = x[r] - p;"),
    "syrk_sign": ("double p = AT(P, ldp, r, i) * AT(P, ldp, r, j);\n                acc = acc - p;",
                  "double p = AT(P, ldp, r, i) * AT(P, ldp, r, j);\n                acc = acc + p;"),
    "gemm_wrong_operand": ("double p = AT(X, ldx, r, i) * AT(Y, ldy, r, j);",
                           "double p = AT(Y, ldy, r, i) * AT(Y, ldy, r, j);"),
    "var2_drops_gemm": ("            oracle_gemm_tn(bk, m, k, A01, lda, A02, lda, A12, lda);\n", ""),
    "var1_drops_syrk": ("            oracle_syrk_upper(bk, k, A01, lda, A11, lda);\n            info = oracle_potrf_upper(bk, A11, lda, 1);\n            if (info) return (int)(k + info);\n        } else {",
                        "            info = oracle_potrf_upper(bk, A11, lda, 1);\n            if (info) return (int)(k + info);\n        } else {"),
    "breakdown_misses_nan": ("if (!(a > 0.0)) {", "if (a <= 0.0) {"),
    "solve_back_transposed": ("double p = AT(U, ldu, r, s) * x[s];", "double p = AT(U, ldu, s, r) * x[s];"),
}


def _pins_pass(L) -> bool:
    """Runs the pin battery against library L; True iff every pin holds."""
    saved = oracle._lib
    oracle._lib = L
    try:
        checks = []
        # exact-arithmetic input
        W, info = oracle.potrf(inputs.minij_scaled(40))
        checks.append(info == 0 and np.array_equal(np.triu(W), inputs.minij_factor(40)))
        # independent library routine
        A = inputs.spd_bbt(60, 1)
        W, info = oracle.potrf(A)
        checks.append(info == 0 and oracle.forward_difference(W, sl.cholesky(A, lower=False)) < 1e-13)
        # blocked variants reproduce the unblocked loop and reconstruct A
        for v in (1, 2, 3):
            W2, i2 = oracle.potrf_blocked(A, 16, v)
            checks.append(i2 == 0 and np.array_equal(np.triu(W2), np.triu(W)))
            checks.append(oracle.factor_backward_error(A, W2) < 1e-14)
        # block operations against scipy / numpy
        g = np.random.Generator(np.random.PCG64(2))
        U = np.asfortranarray(np.triu(g.standard_normal((12, 12))) + 6 * np.eye(12))
        X = np.asfortranarray(g.standard_normal((12, 5)))
        checks.append(np.allclose(oracle.trsm_upper_t(U, X), sl.solve_triangular(U, X, trans="T"), atol=1e-12))
        P = np.asfortranarray(g.standard_normal((6, 9)))
        C = np.asfortranarray(g.standard_normal((9, 9)))
        checks.append(np.allclose(np.triu(oracle.syrk_upper(C, P)), np.triu(C - P.T @ P), atol=1e-12))
        Xg = np.asfortranarray(g.standard_normal((6, 4)))
        checks.append(np.allclose(oracle.gemm_tn(np.asfortranarray(C[:4]), Xg, P), C[:4] - Xg.T @ P, atol=1e-12))
        # breakdown semantics
        B = inputs.spd_bbt(10, 0)
        B[3, 3] = np.nan
        checks.append(oracle.potrf(B)[1] == 4)
        # solve
        Bv = inputs.rhs(60, 2, 0)
        Xs = oracle.solve(np.triu(W), Bv)
        checks.append(oracle.solve_backward_error(A, Xs, Bv) < 1e-14)
        return all(checks)
    finally:
        oracle._lib = saved


def test_real_oracle_passes_battery():
    assert _pins_pass(oracle.lib())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_fails_a_pin(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    mpath = os.path.join(tmp_path, f"oracle_{name}.c")
    with open(mpath, "w") as f:
        f.write(src.replace(old, new))
    lpath = build(mpath, os.path.join(tmp_path, f"liboracle_{name}.so"))
    assert not _pins_pass(oracle.load(lpath))
