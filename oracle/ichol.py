"""Oracle of the paper's own method: level(k) incomplete Cholesky of a sparse
SPD matrix (Sec. "Symbolic factorization", Alg. symb_fact, and the numeric
Cholesky-by-blocks of Sec. "Numeric factorization: Cholesky-by-blocks", here
element by element).  TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``.

Sparse matrices are (n, rp, ci, val) row arrays (CSR): rp int64[n + 1], ci
int32, val float64.  "Upper" arrays hold each row's entries with column >= row.

* ``nd_grid``: a nested dissection ordering of a structured grid (step 1 of
  Alg. symb_fact for the grid inputs): the box is cut at the middle plane of
  its longest side, the plane is the separator, the halves are ordered first,
  then the separator; boxes of at most ``leaf`` points are leaves.  Returns
  the ordering (new index -> old index) and the ranges of the leaves and
  separators in the new numbering, the block boundaries of the 2D layout.
* ``permute_upper``: the upper rows of P A P^T.
* ``fill_pattern`` (O6, C): the level-k pattern by symbolic elimination.
* ``ichol`` (O7, C): the numeric incomplete factorization on that pattern.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import lib


def _p(a: np.ndarray) -> int:
    return a.ctypes.data_as(ctypes.c_void_p).value or 0


def nd_grid(dims: tuple[int, ...], leaf: int = 64, kinds: bool = False):
    """Nested dissection of the grid with sides ``dims`` (point (x, y[, z])
    has natural index x + dims[0] (y + dims[1] z)).  Returns (order, ranges):
    order[new] = old, ranges = [(start, end), ...] in the new numbering, each
    a leaf box or a separator plane, in order; with ``kinds`` also a list of
    booleans, True for the separators."""
    dims = tuple(int(d) for d in dims)
    strides = [1]
    for d in dims[:-1]:
        strides.append(strides[-1] * d)
    order: list[int] = []
    ranges: list[tuple[int, int]] = []
    is_sep: list[bool] = []

    def points(lo, hi):
        axes = [np.arange(lo[a], hi[a]) for a in range(len(dims))]
        mesh = np.meshgrid(*axes, indexing="ij")
        idx = sum(m.astype(np.int64) * s for m, s in zip(mesh, strides))
        # natural order inside the box (x fastest)
        return np.sort(idx.ravel())

    def rec(lo, hi):
        size = int(np.prod([h - l for l, h in zip(lo, hi)]))
        if size == 0:
            return
        if size <= leaf:
            p = points(lo, hi)
            ranges.append((len(order), len(order) + len(p)))
            is_sep.append(False)
            order.extend(p.tolist())
            return
        a = int(np.argmax([h - l for l, h in zip(lo, hi)]))
        mid = (lo[a] + hi[a]) // 2
        left_hi = list(hi); left_hi[a] = mid
        right_lo = list(lo); right_lo[a] = mid + 1
        sep_lo = list(lo); sep_lo[a] = mid
        sep_hi = list(hi); sep_hi[a] = mid + 1
        rec(lo, left_hi)
        rec(right_lo, hi)
        p = points(sep_lo, sep_hi)
        ranges.append((len(order), len(order) + len(p)))
        is_sep.append(True)
        order.extend(p.tolist())

    rec([0] * len(dims), list(dims))
    if kinds:
        return np.asarray(order, dtype=np.int64), ranges, is_sep
    return np.asarray(order, dtype=np.int64), ranges


def permute_upper(n: int, rp: np.ndarray, ci: np.ndarray, val: np.ndarray, order: np.ndarray):
    """Upper rows of B = P A P^T with B[new_i, new_j] = A[order[new_i],
    order[new_j]] from the full symmetric rows of A.  Returns (rp, ci, val),
    each row sorted by column."""
    inv = np.empty(n, dtype=np.int64)
    inv[order] = np.arange(n, dtype=np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    ni, nj = inv[rows], inv[ci.astype(np.int64)]
    keep = ni <= nj
    ni, nj, v = ni[keep], nj[keep], val[keep]
    o = np.lexsort((nj, ni))
    ni, nj, v = ni[o], nj[o], v[o]
    out_rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(out_rp, ni + 1, 1)
    return np.cumsum(out_rp), nj.astype(np.int32), v.astype(np.float64)


def fill_pattern(n: int, arp: np.ndarray, aci: np.ndarray, k: int):
    """O6: (rp, ci, lev) of the level-k pattern of the upper factor of the
    matrix whose upper rows are (arp, aci)."""
    arp = np.ascontiguousarray(arp, dtype=np.int64)
    aci = np.ascontiguousarray(aci, dtype=np.int32)
    cap = max(16, 4 * len(aci))
    while True:
        rp = np.zeros(n + 1, dtype=np.int64)
        ci = np.zeros(cap, dtype=np.int32)
        lev = np.zeros(cap, dtype=np.int32)
        cnt = lib().oracle_fill_pattern(n, _p(arp), _p(aci), int(k), _p(rp), _p(ci), _p(lev), cap)
        if cnt < 0:
            raise MemoryError("oracle_fill_pattern")
        if cnt <= cap:
            return rp, ci[:cnt].copy(), lev[:cnt].copy()
        cap = int(cnt)


def values_on(rp: np.ndarray, ci: np.ndarray, arp: np.ndarray, aci: np.ndarray, aval: np.ndarray) -> np.ndarray:
    """A's upper values scattered onto the pattern (rp, ci) (0 on fill)."""
    n = len(rp) - 1
    val = np.zeros(len(ci), dtype=np.float64)
    for i in range(n):
        cols = ci[rp[i]:rp[i + 1]]
        a_cols = aci[arp[i]:arp[i + 1]]
        pos = np.searchsorted(cols, a_cols)
        val[rp[i] + pos] = aval[arp[i]:arp[i + 1]]
    return val


def ichol(rp: np.ndarray, ci: np.ndarray, val: np.ndarray) -> tuple[np.ndarray, int]:
    """O7: the incomplete factor on the pattern (rp, ci) from A's values
    ``val`` on it; returns (U values, info) on a copy."""
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    out = np.array(val, dtype=np.float64, copy=True)
    info = lib().oracle_ichol_rows(len(rp) - 1, _p(rp), _p(ci), _p(out))
    if info < 0:
        raise ValueError("every row must start with its diagonal")
    return out, int(info)


def to_dense(rp: np.ndarray, ci: np.ndarray, val: np.ndarray) -> np.ndarray:
    """The rows as a dense (Fortran-order) upper-triangular matrix."""
    n = len(rp) - 1
    D = np.zeros((n, n), order="F")
    rows = np.repeat(np.arange(n), np.diff(rp))
    D[rows, ci] = val
    return D


def triangular_apply(rp: np.ndarray, ci: np.ndarray, U: np.ndarray, order: np.ndarray, r: np.ndarray) -> np.ndarray:
    """z = P^T (U^T U)^{-1} P r for the incomplete factor U (rows of the
    ordered matrix) and the ordering order[new] = old: forward substitution
    with U^T, back substitution with U (scipy's sparse triangular solves)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla

    n = len(rp) - 1
    Um = sp.csr_matrix((U, ci, rp), shape=(n, n))
    t = np.asarray(r, dtype=np.float64)[order]
    y = sla.spsolve_triangular(Um.T.tocsr(), t, lower=True)
    zt = sla.spsolve_triangular(Um, y, lower=False)
    z = np.empty(n)
    z[order] = zt
    return z


def pcg(rp: np.ndarray, ci: np.ndarray, val: np.ndarray, b: np.ndarray, precond=None, tol: float = 1e-10,
        max_iter: int = 1000, x0=None):
    """Preconditioned conjugate gradients for A x = b, A given by its full
    symmetric rows (rp, ci, val); ``precond(r)`` returns M^{-1} r (None: M =
    I).  The textbook recurrences: r = b - A x, z = M^{-1} r, p = z; then
    q = A p, alpha = (r, z) / (p, q), x += alpha p, r -= alpha q, stop when
    ||r|| <= tol ||b||, z = M^{-1} r, beta = (r, z)_new / (r, z)_old,
    p = z + beta p.  Returns (x, iterations, ||r|| / ||b||)."""
    import scipy.sparse as sp

    n = len(rp) - 1
    A = sp.csr_matrix((val, ci, rp), shape=(n, n))
    M = precond if precond is not None else (lambda v: v.copy())
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    r = b - A @ x
    nb = float(np.linalg.norm(b))
    if nb == 0.0 or np.linalg.norm(r) <= tol * nb:
        return x, 0, (float(np.linalg.norm(r)) / nb if nb else 0.0)
    z = M(r)
    p = z.copy()
    rz = float(r @ z)
    it = 0
    while it < max_iter:
        q = A @ p
        alpha = rz / float(p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        rel = float(np.linalg.norm(r)) / nb
        if rel <= tol:
            return x, it, rel
        z = M(r)
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, float(np.linalg.norm(r)) / nb
