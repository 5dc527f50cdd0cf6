"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.

This module only builds test matrices; it performs none of the factorization's
arithmetic.  All random numbers come from numpy's PCG64 generator so that a
(seed, shape) pair names the same bytes on every machine.  Matrices are float64,
Fortran (column-major) ordered, exactly symmetric (the upper triangle is
mirrored), so their bytes are also their row-major bytes.

Recipes (the paper fixes none of them; they are the workloads of the dense
Cholesky benchmarks):
  spd_bbt       A = B B^T + n I, B_ij ~ N(0,1) from PCG64(seed) filled in C order
  spd_kappa     A = Q diag(s) Q^T, Q Haar-orthogonal (QR of a Gaussian, seed+1000,
                column signs fixed by sign(diag R)), s_i = kappa^(-i/(n-1))
  rhs           B ~ N(0,1), n x nrhs, seed+2000
  minij_scaled  A_ij = d_i d_j min(i+1, j+1), d_j = 2^((j mod 7) - 3); its
                factor is U_ij = d_j (i <= j), exact in binary floating point
  pascal        A_ij = C(i+j, i); U_ij = C(j, i)
  laplacian1d   tridiag(-1, 2, -1)
  batch         n_i ~ U{lo..hi} (PCG64(seed).integers, endpoint inclusive),
                then each B_i from the same stream and A_i = B_i B_i^T + n_i I
  spd_wishart_shift_torch
                A = B B^T / n + sigma I, B ~ N(0,1) from PCG64(seed), sigma =
                4 / (kappa - 1): the eigenvalues of B B^T / n fill [0, 4]
                (Marchenko-Pastur, square case), so kappa(A) ~ (4 + sigma) /
                sigma = kappa at the cost of one product (the selector's sweep
                shapes; spd_kappa fixes the spectrum exactly but needs a QR)
  qr_matrix     m x n, N(0,1) from PCG64(seed + 3000) in C order, column j
                scaled by kappa^(-j/(n-1)) (the QR workloads)
  selector_shapes
                (n, batch, dtype, kappa): n and batch log-uniform on [64, 32768]
                and [1, 10000], FP64 with probability 3/4, kappa log-uniform on
                [1, 1e6]
"""
from __future__ import annotations

from math import comb

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _symmetrize_upper(A: np.ndarray) -> np.ndarray:
    """Mirror the upper triangle into the lower one (exact symmetry)."""
    T = np.triu(A)
    S = T + np.triu(T, 1).T
    return np.asfortranarray(S)


def gaussian(n: int, m: int, seed: int) -> np.ndarray:
    """n x m N(0,1) matrix, drawn in C order from PCG64(seed)."""
    return _rng(seed).standard_normal((n, m), dtype=np.float64)


def qr_matrix(m: int, n: int, seed: int = 0, kappa: float = 1.0) -> np.ndarray:
    """m x n Fortran-ordered QR input: G ~ N(0,1) from PCG64(seed + 3000) in C
    order, column j scaled by kappa^(-j/(n-1)) (kappa = 1: plain Gaussian;
    otherwise a condition number of roughly kappa times that of G)."""
    G = _rng(seed + 3000).standard_normal((m, n), dtype=np.float64)
    if kappa != 1.0 and n > 1:
        G = G * (float(kappa) ** (-np.arange(n, dtype=np.float64) / (n - 1)))[None, :]
    return np.asfortranarray(G)


def spd_bbt(n: int, seed: int = 0) -> np.ndarray:
    """A = B B^T + n I with B ~ N(0,1) (n x n) from PCG64(seed); kappa <~ 5."""
    B = gaussian(n, n, seed)
    A = B @ B.T
    A[np.diag_indices(n)] += float(n)
    return _symmetrize_upper(A)


def hpd_bbh(n: int, seed: int = 0) -> np.ndarray:
    """Complex Hermitian positive definite A = B B^H + 2n I, B with N(0,1)
    real and imaginary parts (real parts first, then imaginary, from
    PCG64(seed)); exactly Hermitian (the lower triangle mirrors the upper one
    conjugated), real diagonal, kappa <~ 5.  Fortran-ordered complex128."""
    g = _rng(seed)
    B = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    A = B @ B.conj().T
    A[np.diag_indices(n)] = A.diagonal().real + 2.0 * n
    T = np.triu(A)
    return np.asfortranarray(T + np.triu(T, 1).conj().T)


def hpd_exact(n: int, seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """(A, U) with A = U^H U exactly in binary64: U upper triangular with a
    diagonal of powers of two (1, 2, 4) and off-diagonal entries whose real and
    imaginary parts are small integers, so every step of the unblocked complex
    factorization is exact and recovers U bit for bit."""
    g = _rng(seed)
    U = np.triu(g.integers(-3, 4, (n, n)) + 1j * g.integers(-3, 4, (n, n))).astype(np.complex128)
    U[np.diag_indices(n)] = 2.0 ** g.integers(0, 3, n)
    A = U.conj().T @ U  # small integers: exact
    return np.asfortranarray(A), np.asfortranarray(U)


def diag_dominant(n: int, seed: int = 0) -> np.ndarray:
    """Nonsymmetric A = G + 2 (n + 1) I, G ~ N(0,1) from PCG64(seed):
    diagonally dominant by columns (the off-diagonal column sums of |G| stay
    near 0.8 n), so partial pivoting keeps every diagonal pivot and the LU
    without pivoting is the one LAPACK computes.  Fortran-ordered."""
    G = gaussian(n, n, seed)
    return np.asfortranarray(G + float(n + 1) * np.eye(n) * 2.0)


def lu_exact(n: int, seed: int = 0) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(A, L, U) with A = L U exactly in binary64: L unit lower triangular and U
    upper triangular with small integer entries, U's diagonal powers of two,
    so every step of the unblocked LU without pivoting is exact."""
    g = _rng(seed)
    L = np.tril(g.integers(-2, 3, (n, n)), -1).astype(np.float64) + np.eye(n)
    U = np.triu(g.integers(-2, 3, (n, n))).astype(np.float64)
    U[np.diag_indices(n)] = 2.0 ** g.integers(0, 3, n)
    return np.asfortranarray(L @ U), L, U


def spd_bbt_torch(n: int, seed: int, device):
    """Same recipe as spd_bbt, with the product B B^T formed by torch on
    ``device`` (fast at n = 16384).  The bytes can differ from spd_bbt in the
    last bit because the product's summation order differs; both are exactly
    symmetric SPD matrices of the same distribution.  Returns a torch tensor in
    column-major layout (strides (1, n))."""
    import torch

    B = torch.from_numpy(gaussian(n, n, seed)).to(device)
    A = B @ B.T
    del B
    A.diagonal().add_(float(n))
    A = torch.triu(A)
    A = A + torch.triu(A, 1).T
    return A.T.contiguous().T  # symmetric: same bytes, column-major strides


def haar_orthogonal(n: int, seed: int) -> np.ndarray:
    """Q from the QR of an n x n Gaussian with the column signs of
    sign(diag(R)) folded in (Haar-distributed)."""
    G = gaussian(n, n, seed)
    Q, R = np.linalg.qr(G)
    sgn = np.sign(np.diag(R))
    sgn[sgn == 0] = 1.0
    return Q * sgn


def kappa_spectrum(n: int, kappa: float) -> np.ndarray:
    """s_i = kappa^(-i/(n-1)), i = 0..n-1 (1 down to 1/kappa)."""
    if n == 1:
        return np.ones(1)
    return float(kappa) ** (-np.arange(n, dtype=np.float64) / (n - 1))


def spd_kappa(n: int, kappa: float, seed: int = 0) -> np.ndarray:
    """A = Q diag(s) Q^T with condition number kappa (2-norm)."""
    Q = haar_orthogonal(n, seed + 1000)
    s = kappa_spectrum(n, kappa)
    A = (Q * s) @ Q.T
    return _symmetrize_upper(A)


def spd_kappa_torch(n: int, kappa: float, seed: int, device):
    """spd_kappa with the QR and products done by torch on ``device`` (for
    n = 16384).  Column-major torch tensor."""
    import torch

    G = torch.from_numpy(gaussian(n, n, seed + 1000)).to(device)
    Q, R = torch.linalg.qr(G)
    del G
    sgn = torch.sign(torch.diagonal(R))
    sgn[sgn == 0] = 1.0
    del R
    Q.mul_(sgn)
    s = torch.from_numpy(kappa_spectrum(n, kappa)).to(device)
    A = (Q * s) @ Q.T
    del Q
    A = torch.triu(A)
    A = A + torch.triu(A, 1).T
    return A.T.contiguous().T


def spd_wishart_shift_torch(n: int, kappa: float, seed: int, device, dtype=None):
    """A = B B^T / n + sigma I with sigma = 4 / (kappa - 1) (kappa <= 1.01 is
    taken as 1.01), formed on ``device``; column-major, exactly symmetric."""
    import torch

    sigma = 4.0 / (max(float(kappa), 1.01) - 1.0)
    B = torch.from_numpy(gaussian(n, n, seed)).to(device)
    A = B @ B.T
    del B
    A.mul_(1.0 / n)
    A.diagonal().add_(sigma)
    A = torch.triu(A)
    A = A + torch.triu(A, 1).T
    if dtype is not None:
        A = A.to(dtype)
    return A.T.contiguous().T


def selector_shapes(count: int, seed: int) -> list[tuple[int, int, str, float]]:
    """`count` seeded (n, batch, dtype, kappa) shapes for the selector's
    timing sweep."""
    g = _rng(seed)
    out = []
    for _ in range(count):
        n = int(round(np.exp(g.uniform(np.log(64.0), np.log(32768.0)))))
        b = int(round(np.exp(g.uniform(0.0, np.log(10000.0)))))
        dt = "f64" if g.uniform() < 0.75 else "f32"
        kappa = float(10.0 ** g.uniform(0.0, 6.0))
        out.append((n, b, dt, kappa))
    return out


def rhs(n: int, nrhs: int, seed: int = 0) -> np.ndarray:
    """Right-hand sides, n x nrhs N(0,1) from PCG64(seed + 2000), Fortran."""
    return np.asfortranarray(gaussian(nrhs, n, seed + 2000).T)


def minij_scaled(n: int) -> np.ndarray:
    """A_ij = d_i d_j min(i+1, j+1), d_j = 2^((j mod 7) - 3).

    Its Cholesky factor is U_ij = d_j for i <= j: every intermediate of the
    factorization is an integer times a power of two, so FP64, FP32 and BF16
    arithmetic all reproduce it exactly.  The column-dependent scale d makes a
    transposed tile visible."""
    d = 2.0 ** ((np.arange(n) % 7) - 3)
    idx = np.arange(1, n + 1)
    M = np.minimum.outer(idx, idx).astype(np.float64)
    return np.asfortranarray(M * np.outer(d, d))


def minij_factor(n: int) -> np.ndarray:
    """The exact upper factor of minij_scaled(n): U_ij = d_j for i <= j."""
    d = 2.0 ** ((np.arange(n) % 7) - 3)
    return np.asfortranarray(np.triu(np.ones((n, n)) * d[None, :]))


def pascal(n: int) -> np.ndarray:
    """Symmetric Pascal matrix P_ij = C(i+j, i) (exact in FP64 for n <= 29)."""
    return np.asfortranarray(np.array([[float(comb(i + j, i)) for j in range(n)] for i in range(n)]))


def pascal_factor(n: int) -> np.ndarray:
    """Its upper Cholesky factor U_ij = C(j, i)."""
    return np.asfortranarray(np.array([[float(comb(j, i)) if i <= j else 0.0 for j in range(n)]
                                       for i in range(n)]))


def laplacian1d(n: int) -> np.ndarray:
    A = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    return np.asfortranarray(A)


def batch_sizes(count: int, seed: int = 0, lo: int = 16, hi: int = 512) -> np.ndarray:
    """n_i ~ U{lo..hi} (inclusive), int32."""
    return _rng(seed).integers(lo, hi, endpoint=True, size=count).astype(np.int32)


def batch(count: int, seed: int = 0, lo: int = 16, hi: int = 512):
    """(sizes, matrices): n_i ~ U{lo..hi} from PCG64(seed), then, from the same
    stream, B_i (n_i x n_i, C order) one after another and A_i = B_i B_i^T +
    n_i I."""
    g = _rng(seed)
    sizes = g.integers(lo, hi, endpoint=True, size=count).astype(np.int32)
    return sizes, _batch_from(g, sizes)


def batch_torch(count: int, seed: int, device, lo: int = 16, hi: int = 512, dtype=None):
    """The matrices of ``batch(count, seed, lo, hi)`` (same sizes, same B_i
    from the same stream) with each product B_i B_i^T formed by torch on
    ``device``; returns (sizes, list of column-major device tensors).  The
    bytes can differ from ``batch`` in the last bit (summation order)."""
    import torch

    dtype = torch.float64 if dtype is None else dtype
    g = _rng(seed)
    sizes = g.integers(lo, hi, endpoint=True, size=count).astype(np.int32)
    out = []
    for n in sizes:
        n = int(n)
        B = torch.from_numpy(g.standard_normal((n, n), dtype=np.float64)).to(device)
        A = B @ B.T
        A.diagonal().add_(float(n))
        A = torch.triu(A)
        A = A + torch.triu(A, 1).T
        out.append(A.to(dtype).T.contiguous().T)
    return sizes, out


def _batch_from(g, sizes):
    out = []
    for n in sizes:
        n = int(n)
        B = g.standard_normal((n, n), dtype=np.float64)
        A = B @ B.T
        A[np.diag_indices(n)] += float(n)
        out.append(_symmetrize_upper(A))
    return out


def laplacian_grid(dims, stencil: int = 0, shift: float = 0.0):
    """Discrete Laplacian of a structured grid with Dirichlet boundary, full
    symmetric rows (CSR: rp int64[n + 1], ci int32, val float64) in natural
    order (x fastest).  2-D: stencil 5 (default) or 9; 3-D: 7 (default) or 27.
    Off-diagonal entries -1 for every neighbor of the stencil, diagonal the
    number of stencil neighbors (so the matrix is irreducibly diagonally
    dominant, hence SPD) plus ``shift``.  These stand in for the paper's
    sparse test matrices (nnz per row about 5-9 and about 27)."""
    import itertools

    dims = tuple(int(d) for d in dims)
    nd = len(dims)
    if nd not in (2, 3):
        raise ValueError("2-D or 3-D grids")
    stencil = stencil or (5 if nd == 2 else 7)
    if stencil in (5, 7):
        offs = [o for o in itertools.product((-1, 0, 1), repeat=nd) if sum(abs(v) for v in o) == 1]
    elif stencil in (9, 27):
        offs = [o for o in itertools.product((-1, 0, 1), repeat=nd) if any(o)]
    else:
        raise ValueError("stencil 5 / 9 (2-D) or 7 / 27 (3-D)")
    strides = [1]
    for d in dims[:-1]:
        strides.append(strides[-1] * d)
    n = int(np.prod(dims))
    coords = np.stack(np.unravel_index(np.arange(n), dims[::-1])[::-1], axis=1)  # (x, y[, z])
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [np.full(n, float(len(offs)) + shift)]
    for o in offs:
        c = coords + np.asarray(o)
        ok = np.all((c >= 0) & (c < np.asarray(dims)), axis=1)
        src = np.nonzero(ok)[0]
        dst = (c[ok] * np.asarray(strides)).sum(axis=1)
        rows.append(src)
        cols.append(dst)
        vals.append(np.full(len(src), -1.0))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    o = np.lexsort((c, r))
    r, c, v = r[o], c[o], v[o]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, r + 1, 1)
    return np.cumsum(rp), c.astype(np.int32), v.astype(np.float64)
