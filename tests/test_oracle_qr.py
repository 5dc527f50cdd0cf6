"""Pins of O10, Householder QR by the loop of Fig. "dense-chol"'s pattern
(A = Q R, Q a product of reflectors; the conclusion names QR among the
factorizations the pattern carries over to): closed forms, LAPACK's geqrf
through numpy (the same reflector convention, so the packed output agrees
element by element), the uniqueness of R up to row signs against the
Cholesky factor of A^T A (oracle O1), reconstruction and orthogonality, zero
columns, and planted mistakes that each fail a pin."""
import os

import numpy as np
import pytest

import inputs
import oracle
from oracle.build import SRC, build


def test_two_by_one_closed_form():
    # x = [3, 4]: beta = -5, tau = (-5 - 3) / -5, v = [1, 4 / 8]
    W, tau = oracle.geqrf(np.asfortranarray([[3.0], [4.0]]))
    assert W[0, 0] == -5.0 and W[1, 0] == 0.5
    assert tau[0] == np.float64(-8.0) / np.float64(-5.0)


def test_negative_alpha_closed_form():
    # x = [-3, 4]: beta = +5, tau = (5 + 3) / 5, v = [1, 4 / -8]
    W, tau = oracle.geqrf(np.asfortranarray([[-3.0], [4.0]]))
    assert W[0, 0] == 5.0 and W[1, 0] == -0.5
    assert tau[0] == np.float64(8.0) / np.float64(5.0)


@pytest.mark.parametrize("A", [np.eye(5), -np.eye(5), np.diag([2.0, -3.0, 0.0, 7.0])])
def test_diagonal_input_is_its_own_r(A):
    # no entries below the diagonal: every reflector is the identity
    W, tau = oracle.geqrf(np.asfortranarray(A))
    assert np.array_equal(W, A) and np.array_equal(tau, np.zeros(A.shape[1]))


@pytest.mark.parametrize("m,n", [(1, 1), (6, 1), (40, 40), (97, 64), (200, 130), (300, 257)])
def test_against_lapack_geqrf(m, n):
    A = inputs.qr_matrix(m, n, seed=m + n)
    W, tau = oracle.geqrf(A)
    h, tl = np.linalg.qr(A, mode="raw")  # LAPACK geqrf: h is the packed result, transposed
    scale = np.max(np.abs(A))
    assert np.max(np.abs(W - h.T)) <= 1e-13 * scale * np.sqrt(m)
    assert np.max(np.abs(tau - tl)) <= 1e-13


@pytest.mark.parametrize("m,n", [(50, 50), (120, 80)])
def test_r_is_cholesky_of_gram_up_to_row_signs(m, n):
    A = inputs.qr_matrix(m, n, seed=7)
    W, tau = oracle.geqrf(A)
    R = np.triu(W[:n, :])
    C, info = oracle.potrf(np.asfortranarray(A.T @ A))
    assert info == 0
    D = np.sign(np.diag(R))
    assert np.all(D != 0)
    assert np.max(np.abs(D[:, None] * R - np.triu(C))) <= 1e-11 * np.max(np.abs(R))


@pytest.mark.parametrize("m,n,kappa", [(64, 64, 1.0), (150, 100, 1.0), (128, 128, 1e8)])
def test_reconstruction_and_orthogonality(m, n, kappa):
    A = inputs.qr_matrix(m, n, seed=3, kappa=kappa)
    W, tau = oracle.geqrf(A)
    assert oracle.qr_backward_error(A, W, tau) <= 1e-15 * np.sqrt(m) * 10
    assert oracle.qr_orthogonality(W, tau) <= 1e-15 * m


def test_zero_column_gives_identity_reflector():
    A = inputs.qr_matrix(30, 10, seed=1)
    A[:, 4] = 0.0
    W, tau = oracle.geqrf(A)
    # after the first four reflectors column 4 is still zero: tau_4 = 0
    assert tau[4] == 0.0 and np.all(W[4:, 4] == 0.0)
    assert oracle.qr_backward_error(A, W, tau) <= 1e-14


MUTANTS = {
    "qr_beta_sign": ("double beta = alpha >= 0.0 ? -mag : mag;", "double beta = alpha >= 0.0 ? mag : -mag;"),
    "qr_tau_sign": ("double tj = (beta - alpha) / beta;", "double tj = (alpha - beta) / beta;"),
    "qr_w_drops_top": ("double w = AT(A, lda, j, c);", "double w = 0.0;"),
    "qr_update_skips_last_row": ("for (int64_t i = j + 1; i < m; ++i) AT(A, lda, i, c)",
                                 "for (int64_t i = j + 1; i < m - 1; ++i) AT(A, lda, i, c)"),
    "qr_sigma_includes_alpha": ("for (int64_t r = j + 1; r < m; ++r) sigma += AT(A, lda, r, j) * AT(A, lda, r, j);",
                                "for (int64_t r = j; r < m; ++r) sigma += AT(A, lda, r, j) * AT(A, lda, r, j);"),
}


def _pins_pass(L) -> bool:
    saved = oracle._lib
    oracle._lib = L
    try:
        checks = []
        W, tau = oracle.geqrf(np.asfortranarray([[3.0], [4.0]]))
        checks.append(W[0, 0] == -5.0 and W[1, 0] == 0.5 and tau[0] == np.float64(-8.0) / np.float64(-5.0))
        A = inputs.qr_matrix(97, 64, seed=161)
        W, tau = oracle.geqrf(A)
        h, tl = np.linalg.qr(A, mode="raw")
        checks.append(np.max(np.abs(W - h.T)) <= 1e-12 and np.max(np.abs(tau - tl)) <= 1e-13)
        checks.append(oracle.qr_backward_error(A, W, tau) <= 1e-14)
        return all(checks)
    finally:
        oracle._lib = saved


def test_real_oracle_passes_qr_battery():
    assert _pins_pass(oracle.lib())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_qr_mutant_fails_a_pin(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    mpath = os.path.join(tmp_path, f"oracle_{name}.c")
    with open(mpath, "w") as f:
        f.write(src.replace(old, new))
    lpath = build(mpath, os.path.join(tmp_path, f"liboracle_{name}.so"))
    assert not _pins_pass(oracle.load(lpath))
