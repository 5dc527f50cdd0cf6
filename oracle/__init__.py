"""FP64 CPU oracle for the dense blocked Cholesky A = U^T U (arXiv 1601.05871,
Fig. "dense-chol").

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the library.  It shares no
code with the GPU path.  The arithmetic lives in ``oracle.c`` (plain loops,
FP64, no contraction); this module marshals numpy arrays into it and adds the
accuracy metrics (plain numpy in FP64).

Every matrix is a 2-D numpy float64 array in column-major (Fortran) order;
only its upper triangle is read or written by the factor routines.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import build as _build, LIB_PATH

_lib = None


def load(path: str) -> ctypes.CDLL:
    """Load an oracle shared library and declare its signatures."""
    L = ctypes.CDLL(path)
    if True:
        i64, i32, dp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        L.oracle_potrf_upper.argtypes = [i64, dp, i64, i32]
        L.oracle_potrf_upper.restype = i32
        L.oracle_potrf_upper_steps.argtypes = [i64, dp, i64, i64, i32]
        L.oracle_potrf_upper_steps.restype = i32
        L.oracle_potrf_blocked.argtypes = [i64, dp, i64, i64, i32, i64]
        L.oracle_potrf_blocked.restype = i32
        L.oracle_trsm_upper_t.argtypes = [i64, i64, dp, i64, dp, i64]
        L.oracle_trsm_upper_t.restype = None
        L.oracle_syrk_upper.argtypes = [i64, i64, dp, i64, dp, i64]
        L.oracle_syrk_upper.restype = None
        L.oracle_gemm_tn.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, i64]
        L.oracle_gemm_tn.restype = None
        L.oracle_solve_upper.argtypes = [i64, i64, dp, i64, dp, i64]
        L.oracle_solve_upper.restype = None
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = i32
        L.oracle_fill_pattern.argtypes = [i64, dp, dp, i32, dp, dp, dp, i64]
        L.oracle_fill_pattern.restype = i64
        L.oracle_ichol_rows.argtypes = [i64, dp, dp, dp]
        L.oracle_ichol_rows.restype = i32
        L.oracle_zpotrf_upper.argtypes = [i64, dp, i64]
        L.oracle_zpotrf_upper.restype = i32
        L.oracle_getrf_nopiv.argtypes = [i64, dp, i64]
        L.oracle_getrf_nopiv.restype = i32
        L.oracle_geqrf.argtypes = [i64, i64, dp, i64, dp]
        L.oracle_geqrf.restype = None
    return L


def lib() -> ctypes.CDLL:
    """Load liboracle.so, compiling it first if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            _build()
        _lib = load(LIB_PATH)
    return _lib


def _fortran(a: np.ndarray) -> np.ndarray:
    if a.dtype != np.float64 or a.ndim != 2 or not a.flags.f_contiguous:
        raise TypeError("oracle expects a 2-D float64 Fortran-ordered array")
    return a


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _ld(a: np.ndarray) -> int:
    # leading dimension of a Fortran-ordered array (also for column slices)
    return a.strides[1] // 8 if a.shape[1] > 1 else max(1, a.shape[0])


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def potrf(A: np.ndarray, threads: int = 1, steps: int | None = None) -> tuple[np.ndarray, int]:
    """O1: unblocked Cholesky (Fig. "dense-chol" at b = 1) on a copy of A.

    Returns (A_out, info).  A_out's upper triangle holds U (or, if ``steps`` is
    given, the first ``steps`` rows of U above the Schur complement); its
    strictly lower triangle is A's, untouched.  info = 0 on success, else the
    1-based column of the first pivot that is not > 0.
    """
    W = np.array(_fortran(A), dtype=np.float64, order="F", copy=True)
    n = W.shape[0]
    js = n if steps is None else int(steps)
    info = lib().oracle_potrf_upper_steps(n, _ptr(W), max(1, n), js, int(threads))
    return W, int(info)


def zpotrf(A: np.ndarray) -> tuple[np.ndarray, int]:
    """O8: unblocked complex Cholesky A = U^H U (Fig. "dense-chol" at b = 1
    with the Hermitian update) on a copy of the complex128 matrix A.
    Returns (A_out, info) as :func:`potrf`: the upper triangle holds U (real
    positive diagonal), the strictly lower triangle is A's, untouched."""
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise TypeError("zpotrf expects a square matrix")
    W = np.array(A, dtype=np.complex128, order="F", copy=True)
    n = W.shape[0]
    info = lib().oracle_zpotrf_upper(n, _ptr(W), max(1, n))
    return W, int(info)


def getrf_nopiv(A: np.ndarray) -> tuple[np.ndarray, int]:
    """O9: LU without pivoting, A = L U, on a copy of A: the strictly lower
    triangle receives L (unit diagonal implied), the upper triangle U.
    Returns (A_out, info); info = first zero or non-finite pivot (1-based)."""
    W = np.array(_fortran(A), dtype=np.float64, order="F", copy=True)
    n = W.shape[0]
    info = lib().oracle_getrf_nopiv(n, _ptr(W), max(1, n))
    return W, int(info)


def lu_backward_error(A: np.ndarray, W: np.ndarray) -> float:
    """||A - L U||_F / ||A||_F for the packed factors W of :func:`getrf_nopiv`."""
    n = W.shape[0]
    L = np.tril(W, -1) + np.eye(n)
    U = np.triu(W)
    return float(np.linalg.norm(A - L @ U) / np.linalg.norm(A))


def geqrf(A: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """O10: Householder QR of the m x n (m >= n) matrix A on a copy: R in the
    upper triangle, the reflectors' vectors below the diagonal (unit entry
    implied), and their scalars tau (n).  Q = H_0 ... H_{n-1},
    H_j = I - tau_j v_j v_j^T."""
    W = np.array(_fortran(A), dtype=np.float64, order="F", copy=True)
    m, n = W.shape
    tau = np.zeros(n, dtype=np.float64)
    lib().oracle_geqrf(m, n, _ptr(W), max(1, m), _ptr(tau))
    return W, tau


def qr_form_q(W: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """The m x n matrix Q[:, :n] of the packed reflectors (W, tau) of
    :func:`geqrf`: H_0 ... H_{n-1} applied to the first n columns of I, the
    last reflector first."""
    m, n = W.shape
    Q = np.eye(m, n)
    for j in range(n - 1, -1, -1):
        v = np.zeros(m)
        v[j] = 1.0
        v[j + 1:] = W[j + 1:, j]
        Q -= tau[j] * np.outer(v, v @ Q)
    return Q


def qr_backward_error(A: np.ndarray, W: np.ndarray, tau: np.ndarray) -> float:
    """||A - Q R||_F / ||A||_F for the packed QR factors (W, tau)."""
    Q = qr_form_q(W, tau)
    return float(np.linalg.norm(A - Q @ np.triu(W[: W.shape[1], :])) / np.linalg.norm(A))


def qr_orthogonality(W: np.ndarray, tau: np.ndarray) -> float:
    """||Q^T Q - I||_F for the first n columns of Q."""
    Q = qr_form_q(W, tau)
    return float(np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1])))


def zfactor_backward_error(A: np.ndarray, U: np.ndarray) -> float:
    """||A - U^H U||_F / ||A||_F for the upper triangle U of a complex factor
    (A Hermitian, given by its upper triangle)."""
    Ah = np.triu(A) + np.triu(A, 1).conj().T
    Ut = np.triu(U)
    return float(np.linalg.norm(Ah - Ut.conj().T @ Ut) / np.linalg.norm(Ah))


def potrf_inplace(W: np.ndarray, lda: int, n: int, threads: int = 0, steps: int | None = None) -> int:
    """O1 in place on a Fortran buffer (used for timing the oracle)."""
    js = n if steps is None else int(steps)
    return int(lib().oracle_potrf_upper_steps(n, _ptr(W), lda, js, int(threads)))


def potrf_blocked(A: np.ndarray, b: int, variant: int, iters: int = -1) -> tuple[np.ndarray, int]:
    """O2: the blocked loop of Fig. "dense-chol" for loop invariant
    ``variant`` (1 bordered, 2 left-looking, 3 right-looking) on a copy of A."""
    W = np.array(_fortran(A), dtype=np.float64, order="F", copy=True)
    n = W.shape[0]
    info = lib().oracle_potrf_blocked(n, _ptr(W), max(1, n), int(b), int(variant), int(iters))
    return W, int(info)


def trsm_upper_t(U: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Returns triu(U)^{-T} X (the TRSM step of Fig. "dense-chol")."""
    U = np.asfortranarray(U, dtype=np.float64)
    Y = np.array(X, dtype=np.float64, order="F", copy=True)
    b, m = Y.shape
    lib().oracle_trsm_upper_t(b, m, _ptr(U), max(1, U.shape[0]), _ptr(Y), max(1, b))
    return Y


def syrk_upper(C: np.ndarray, P: np.ndarray) -> np.ndarray:
    """Returns C - P^T P on the upper triangle (the HERK step); C's strictly
    lower triangle is returned unchanged."""
    P = np.asfortranarray(P, dtype=np.float64)
    D = np.array(C, dtype=np.float64, order="F", copy=True)
    k, m = P.shape
    lib().oracle_syrk_upper(m, k, _ptr(P), max(1, k), _ptr(D), max(1, m))
    return D


def gemm_tn(C: np.ndarray, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Returns C - X^T Y (the off-diagonal block form of the HERK step)."""
    X = np.asfortranarray(X, dtype=np.float64)
    Y = np.asfortranarray(Y, dtype=np.float64)
    D = np.array(C, dtype=np.float64, order="F", copy=True)
    k, mr = X.shape
    nc = Y.shape[1]
    lib().oracle_gemm_tn(mr, nc, k, _ptr(X), max(1, k), _ptr(Y), max(1, k), _ptr(D), max(1, mr))
    return D


def solve(U: np.ndarray, B: np.ndarray) -> np.ndarray:
    """O3: X with U^T U X = B (forward then back substitution)."""
    U = np.asfortranarray(U, dtype=np.float64)
    X = np.array(B, dtype=np.float64, order="F", copy=True)
    if X.ndim == 1:
        X = X.reshape(-1, 1, order="F")
    n, nrhs = X.shape
    lib().oracle_solve_upper(n, nrhs, _ptr(U), max(1, U.shape[0]), _ptr(X), max(1, n))
    return X


# ----------------------------------------------------------------------------
# Cholesky-by-blocks over a block pattern (Fig. "sparse-chol" with dense
# blocks), composed of the oracle's block operations above.

def chol_by_blocks(A: np.ndarray, pattern=None, b: int = 128) -> tuple[np.ndarray, int]:
    """The loop of Fig. "sparse-chol" on blocks of order b (the last ones
    ragged): for each k, CHOL of the diagonal block, TRSM of every existing
    block of block row k, then for every pair i <= j of existing blocks of that
    row the HERK / GEMM update of block (i, j) if that block exists (the
    exist(A22(i, j)) filter; an update of a missing block is dropped).
    ``pattern``: nbt x nbt boolean array, True = block (i, j) exists (upper
    triangle read; diagonal always exists); None = dense.  Blocks that do not
    exist are left as they are.  Returns (A_out, info) on a copy; info as potrf
    (1-based column of the first non-positive pivot).  Pinned (tests): a dense
    pattern gives O1 bit for bit; a pattern closed under fill recovers U from
    A = U^T U; with fill dropped, U^T U equals A on every existing block (the
    defining property of the block incomplete factor)."""
    W = np.array(_fortran(A), dtype=np.float64, order="F", copy=True)
    n = W.shape[0]
    nbt = (n + b - 1) // b

    def ex(i, j):
        return i == j or pattern is None or bool(pattern[i][j])

    def sl(i):
        return slice(i * b, min(n, (i + 1) * b))

    for k in range(nbt):
        Ukk, info = potrf(np.asfortranarray(W[sl(k), sl(k)]))
        W[sl(k), sl(k)] = np.triu(Ukk) + np.tril(W[sl(k), sl(k)], -1)
        if info:
            return W, k * b + info
        row = [j for j in range(k + 1, nbt) if ex(k, j)]
        for j in row:
            W[sl(k), sl(j)] = trsm_upper_t(np.triu(W[sl(k), sl(k)]), np.asfortranarray(W[sl(k), sl(j)]))
        for i in row:
            for j in row:
                if j < i or not ex(i, j):
                    continue
                Xi = np.asfortranarray(W[sl(k), sl(i)])
                Yj = np.asfortranarray(W[sl(k), sl(j)])
                C = np.asfortranarray(W[sl(i), sl(j)])
                if i == j:
                    W[sl(i), sl(j)] = syrk_upper(C, Xi)
                else:
                    W[sl(i), sl(j)] = gemm_tn(C, Xi, Yj)
    return W, 0


# ----------------------------------------------------------------------------
# Metrics (O4), FP64 numpy.  U is read from the upper triangle only.

def upper(M: np.ndarray) -> np.ndarray:
    return np.triu(M)


def sym_from_upper(A: np.ndarray) -> np.ndarray:
    """The symmetric matrix whose upper triangle is A's."""
    T = np.triu(A)
    return T + np.triu(T, 1).T


def factor_backward_error(A: np.ndarray, U: np.ndarray) -> float:
    """beta_F = ||A - U^T U||_F / ||A||_F, with A symmetric from its upper part."""
    S = sym_from_upper(A)
    Uu = np.triu(U)
    R = S - Uu.T @ Uu
    return float(np.linalg.norm(R) / np.linalg.norm(S))


def factor_backward_error_est(A: np.ndarray, U: np.ndarray, seed: int = 0, k: int = 8) -> float:
    """Randomized estimate ||(A - U^T U) X||_F / (||A||_F ||X||_F), X n x k
    N(0,1), computed as A X - U^T (U X) in O(n^2 k) (used where n is too large
    for the exact norm).  A is symmetric from its upper triangle."""
    n = A.shape[0]
    X = np.random.Generator(np.random.PCG64(seed)).standard_normal((n, k))
    Au = np.triu(A)
    AX = Au @ X + np.triu(A, 1).T @ X
    Uu = np.triu(U)
    R = AX - Uu.T @ (Uu @ X)
    nA = np.sqrt(2.0 * np.sum(Au * Au) - np.sum(np.diag(A) ** 2))
    return float(np.linalg.norm(R) / (nA * np.linalg.norm(X)))


def solve_backward_error(A: np.ndarray, X: np.ndarray, B: np.ndarray) -> float:
    """Normwise backward error eta = ||b - A x||_inf / (||A||_inf ||x||_inf +
    ||b||_inf), the maximum over the columns; A symmetric from its upper part."""
    S = sym_from_upper(A)
    X = X.reshape(X.shape[0], -1)
    B = B.reshape(B.shape[0], -1)
    R = B - S @ X
    nA = np.max(np.sum(np.abs(S), axis=1))
    eta = 0.0
    for c in range(X.shape[1]):
        den = nA * np.max(np.abs(X[:, c])) + np.max(np.abs(B[:, c]))
        eta = max(eta, float(np.max(np.abs(R[:, c])) / den))
    return eta


def forward_difference(U_hat: np.ndarray, U_ref: np.ndarray) -> float:
    """||U_hat - U_ref||_F / ||U_ref||_F over the upper triangles."""
    D = np.triu(U_hat) - np.triu(U_ref)
    return float(np.linalg.norm(D) / np.linalg.norm(np.triu(U_ref)))


def flops(n: int) -> float:
    """Algorithmic flop count of a Cholesky factorization (LAPACK potrf count):
    n^3/3 + n^2/2 + n/6 = n(n+1)(2n+1)/6."""
    n = int(n)
    return float(n * (n + 1) * (2 * n + 1) // 6)
