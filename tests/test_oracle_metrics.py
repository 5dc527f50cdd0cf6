"""Known-value pins of the oracle's accuracy metrics (O4) and mutants of them.

Each pin is a tiny system whose metric is worked out by hand in exact
arithmetic (the comment beside it shows the arithmetic), so it checks the
definitions themselves, not a retyped formula:

  factor backward error  beta_F = ||A - U^T U||_F / ||A||_F   (reconstruction
                         A = U^T U of the dense Cholesky figure)
  randomized estimate    ||(A - U^T U) X||_F / (||A||_F ||X||_F)
  solve backward error   eta = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf)
                         (normwise, Rigal-Gaches), max over columns
  forward difference     ||U_hat - U_ref||_F / ||U_ref||_F

Only upper triangles are meaningful: every pin also plants garbage in the
strictly lower triangles, which must not change the value.

The mutants plant plausible mistakes (a squared norm, a 1-norm for an
infinity norm, a dropped term, a transposed factor, reading the lower
triangle) in a copy of the metric source; each must fail at least one pin.
"""
import inspect
import math

import numpy as np
import pytest

import oracle

GARBAGE = 1e3


def _f(rows):
    return np.asfortranarray(np.array(rows, dtype=np.float64))


def _with_lower_garbage(M, value=GARBAGE):
    M = M.copy(order="F")
    il = np.tril_indices(M.shape[0], -1, M.shape[1])
    M[il] = value
    return M


# ---- pins ------------------------------------------------------------------

def pin_factor_backward_error(fns):
    # A = [[4, 2], [2, 5]] has U = [[2, 1], [0, 2]].  With U_hat(1,1) = 2.5:
    # U_hat^T U_hat = [[4, 2], [2, 1 + 6.25]], so A - U_hat^T U_hat =
    # [[0, 0], [0, -2.25]]; ||A||_F = sqrt(16 + 4 + 4 + 25) = 7 => 2.25 / 7.
    A = _with_lower_garbage(_f([[4, 2], [2, 5]]))
    U = _with_lower_garbage(_f([[2, 1], [0, 2.5]]))
    ok = [abs(fns["factor_backward_error"](A, U) - 2.25 / 7) <= 1e-15]
    # the exact factor: zero
    ok.append(fns["factor_backward_error"](A, _with_lower_garbage(_f([[2, 1], [0, 2]]))) == 0.0)
    # an off-diagonal residual: U_hat = [[2, 1.5], [0, u]], u^2 = 5 - 2.25:
    # A - U_hat^T U_hat = [[0, -1], [-1, 0]] (up to the rounding of u) =>
    # sqrt(2) / 7
    U2 = _with_lower_garbage(_f([[2, 1.5], [0, math.sqrt(2.75)]]))
    ok.append(abs(fns["factor_backward_error"](A, U2) - math.sqrt(2) / 7) <= 1e-15)
    return all(ok)


def pin_factor_backward_error_est(fns):
    # A - U^T U = E with E orthogonal up to a scalar e gives ||E X||_F =
    # e ||X||_F for every X, so the estimate equals e / ||A||_F exactly.
    ok = []
    # A = 5 I_4, U = 2 I_4: E = I, ||A||_F = 10 => 0.1
    A = _with_lower_garbage(np.asfortranarray(5.0 * np.eye(4)))
    U = _with_lower_garbage(np.asfortranarray(2.0 * np.eye(4)))
    ok.append(abs(fns["factor_backward_error_est"](A, U, seed=3) - 0.1) <= 1e-15)
    # A = [[4, 2], [2, 5]], U_hat = [[2, 1.5], [0, sqrt(2.75)]]: E = -[[0, 1], [1, 0]]
    # (a permutation), ||A||_F = 7 => 1 / 7
    A2 = _with_lower_garbage(_f([[4, 2], [2, 5]]))
    U2 = _with_lower_garbage(_f([[2, 1.5], [0, math.sqrt(2.75)]]))
    for seed in (0, 1):
        ok.append(abs(fns["factor_backward_error_est"](A2, U2, seed=seed) - 1 / 7) <= 1e-15)
    return all(ok)


def pin_solve_backward_error(fns):
    # A = [[2, 1], [1, 3]], x = [1, 2]: A x = [4, 7].  b = [5, 8] => r = [1, 1],
    # ||r||_inf = 1, ||A||_inf = 4, ||x||_inf = 2, ||b||_inf = 8 => 1 / 16.
    A = _with_lower_garbage(_f([[2, 1], [1, 3]]))
    x = _f([[1], [2]])
    b = _f([[5], [8]])
    ok = [abs(fns["solve_backward_error"](A, x, b) - 1 / 16) <= 1e-16]
    # a second column with the larger error: x = [0, 1], A x = [1, 3],
    # b = [3, 3] => r = [2, 0]; 2 / (4 * 1 + 3) = 2 / 7; the max is 2 / 7
    X = _f([[1, 0], [2, 1]])
    B = _f([[5, 3], [8, 3]])
    ok.append(abs(fns["solve_backward_error"](A, X, B) - 2 / 7) <= 1e-16)
    # an exact solution: zero
    ok.append(fns["solve_backward_error"](A, x, _f([[4], [7]])) == 0.0)
    return all(ok)


def pin_forward_difference(fns):
    # U_hat - U_ref = [[0, 1], [0, 0]], ||U_ref||_F = sqrt(4 + 4) => 1 / sqrt(8)
    Uh = _with_lower_garbage(_f([[2, 1], [0, 2]]))
    Ur = _with_lower_garbage(_f([[2, 0], [0, 2]]), value=-7 * GARBAGE)
    return abs(fns["forward_difference"](Uh, Ur) - 1 / math.sqrt(8)) <= 1e-16


PINS = (pin_factor_backward_error, pin_factor_backward_error_est, pin_solve_backward_error,
        pin_forward_difference)
METRICS = ("sym_from_upper", "factor_backward_error", "factor_backward_error_est", "solve_backward_error",
           "forward_difference")


def _real_fns():
    return {k: getattr(oracle, k) for k in METRICS}


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_metric_pin(pin):
    assert pin(_real_fns())


# ---- mutants ------------------------------------------------------------------

MUTANTS = {
    # factor_backward_error
    "beta_squared_norm": ("return float(np.linalg.norm(R) / np.linalg.norm(S))",
                          "return float(np.linalg.norm(R) / np.linalg.norm(S) ** 2)"),
    "beta_untransposed": ("R = S - Uu.T @ Uu", "R = S - Uu @ Uu.T"),
    "beta_full_U": ("    Uu = np.triu(U)\n    R = S - Uu.T @ Uu", "    Uu = U\n    R = S - Uu.T @ Uu"),
    "sym_reads_lower": ("return T + np.triu(T, 1).T", "return T + np.tril(A, -1)"),
    # factor_backward_error_est
    "est_drops_diag_term": ("nA = np.sqrt(2.0 * np.sum(Au * Au) - np.sum(np.diag(A) ** 2))",
                            "nA = np.sqrt(2.0 * np.sum(Au * Au))"),
    "est_upper_only": ("AX = Au @ X + np.triu(A, 1).T @ X", "AX = Au @ X"),
    "est_no_x_norm": ("return float(np.linalg.norm(R) / (nA * np.linalg.norm(X)))",
                      "return float(np.linalg.norm(R) / nA)"),
    # solve_backward_error
    "eta_one_norm_r": ("eta = max(eta, float(np.max(np.abs(R[:, c])) / den))",
                       "eta = max(eta, float(np.sum(np.abs(R[:, c])) / den))"),
    "eta_one_norm_x": ("den = nA * np.max(np.abs(X[:, c])) + np.max(np.abs(B[:, c]))",
                       "den = nA * np.sum(np.abs(X[:, c])) + np.max(np.abs(B[:, c]))"),
    "eta_drops_b": ("den = nA * np.max(np.abs(X[:, c])) + np.max(np.abs(B[:, c]))",
                    "den = nA * np.max(np.abs(X[:, c]))"),
    "eta_frobenius_A": ("nA = np.max(np.sum(np.abs(S), axis=1))", "nA = np.linalg.norm(S)"),
    "eta_first_column_only": ("for c in range(X.shape[1]):", "for c in range(1):"),
    # forward_difference
    "fwd_full_matrices": ("D = np.triu(U_hat) - np.triu(U_ref)", "D = U_hat - U_ref"),
    "fwd_absolute": ("return float(np.linalg.norm(D) / np.linalg.norm(np.triu(U_ref)))",
                     "return float(np.linalg.norm(D))"),
}


def _mutated_fns(old: str, new: str):
    src = "\n\n".join(inspect.getsource(getattr(oracle, k)) for k in METRICS)
    assert src.count(old) == 1, f"mutation site not unique: {old!r}"
    ns = {"np": np}
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    return {k: ns[k] for k in METRICS}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_metric_mutant_fails_a_pin(name):
    fns = _mutated_fns(*MUTANTS[name])
    assert not all(p(fns) for p in PINS)
