"""Complex Hermitian factorization (flame_factor with dtype FLAME_Z64,
A = U^H U) against the complex oracle O8, element by element: ragged orders
across the 64-blocks of the LDS kernels and the outer blocks, padded leading
dimensions, lower storage, breakdown, the untouched triangle."""
import ctypes

import numpy as np
import pytest
import torch

import inputs
import oracle
import paper_1601_05871_amd as fl
from gpu_util import DEV

pytestmark = pytest.mark.gpu


def _dev(A: np.ndarray, ld: int):
    """Column-major complex128 device copy with leading dimension ld (padding
    rows NaN)."""
    n = A.shape[0]
    base = torch.full((max(n, 1) * ld,), complex(float("nan"), float("nan")), dtype=torch.complex128, device=DEV)
    T = base.as_strided((n, n), (1, ld))
    if n:
        T.copy_(torch.from_numpy(np.asarray(A, dtype=np.complex128)))
    return base, T


def _host(T) -> np.ndarray:
    torch.cuda.synchronize()
    return np.asfortranarray(T.cpu().numpy())


@pytest.mark.parametrize("n,nb,pad", [(1, 64, 0), (2, 64, 1), (17, 64, 0), (63, 64, 2), (64, 64, 0), (65, 64, 0),
                                      (127, 128, 3), (128, 128, 0), (129, 64, 0), (200, 128, 5), (300, 256, 0),
                                      (513, 256, 1), (700, 512, 0)])
def test_complex_matches_oracle(n, nb, pad):
    print(f"[complex] n={n} nb={nb} pad={pad}", flush=True)
    A = inputs.hpd_bbh(n, 100 + n)
    Uo, io = oracle.zpotrf(A)
    base, T = _dev(A, n + pad)
    info = fl.factor(T, variant=fl.VAR_RIGHT, nb=nb)
    W = _host(T)
    assert int(info.item()) == io == 0
    U = np.triu(W)
    assert np.max(np.abs(U - np.triu(Uo))) <= 1e-13 * np.max(np.abs(Uo))
    assert oracle.zfactor_backward_error(A, W) <= 1e-14
    assert np.all(np.diag(W).imag == 0)
    il = np.tril_indices(n, -1)
    assert np.array_equal(W[il], A[il])  # strictly lower triangle untouched
    if pad:
        full = base.cpu().numpy()[: n * (n + pad)].reshape(n, n + pad).T
        assert np.all(np.isnan(full[n:]))  # padding rows never written


@pytest.mark.parametrize("n", [20, 64])
def test_complex_exact_factor_recovered(n):
    """Integer factor with power-of-two diagonal, one diagonal block (the LDS
    kernel alone): every step is exact, so the device recovers U bit for bit.
    (These factors are far too ill-conditioned for larger orders: the panel
    solve's block inverses are not exact there.)"""
    A, U = inputs.hpd_exact(n, 7)
    _, T = _dev(A, n)
    assert int(fl.factor(T, variant=fl.VAR_RIGHT, nb=64).item()) == 0
    assert np.array_equal(np.triu(_host(T)), U)


def test_complex_real_input_matches_real_path():
    n = 400
    A = inputs.spd_bbt(n, 9)
    _, T = _dev(A.astype(np.complex128), n)
    assert int(fl.factor(T, variant=fl.VAR_RIGHT, nb=128).item()) == 0
    W = _host(T)
    Ur, _ = oracle.potrf(A, threads=8)
    assert np.max(np.abs(np.triu(W).real - np.triu(Ur))) <= 1e-13 * np.max(np.abs(Ur))
    assert np.max(np.abs(np.triu(W).imag)) <= 1e-14 * np.max(np.abs(Ur))


@pytest.mark.parametrize("n,nb", [(90, 64), (333, 128)])
def test_complex_lower_storage(n, nb):
    A = inputs.hpd_bbh(n, 40 + n)
    Uo, _ = oracle.zpotrf(A)
    M = np.array(A, order="F", copy=True)
    iu = np.triu_indices(n, 1)
    M[iu] = 7.0 - 3.0j  # the strictly upper triangle is not part of the input
    _, T = _dev(M, n)
    assert int(fl.factor(T, variant=fl.VAR_RIGHT, nb=nb, lower=True).item()) == 0
    W = _host(T)
    L = np.tril(W)
    assert np.max(np.abs(L - np.triu(Uo).conj().T)) <= 1e-13 * np.max(np.abs(Uo))  # A = L L^H, L = U^H
    assert np.all(W[iu] == 7.0 - 3.0j)


def test_complex_breakdown_column():
    n = 260
    A = inputs.hpd_bbh(n, 3)
    A[190, 190] = -4.0 * n
    _, io = oracle.zpotrf(A)
    assert io > 0
    _, T = _dev(A, n)
    assert int(fl.factor(T, variant=fl.VAR_RIGHT, nb=128).item()) == io


def test_complex_sampled_large():
    """n = 2048 at the default block (256): every element of the first and
    last 64 columns of U against the oracle, and the backward error."""
    n = 2048
    A = inputs.hpd_bbh(n, 11)
    Uo, io = oracle.zpotrf(A)
    _, T = _dev(A, n)
    info = torch.zeros(1, dtype=torch.int32, device=DEV)
    o = fl.Opts(fl.VAR_RIGHT, 0, 0, 0, 0, 0)
    rc = fl.lib().flame_factor(fl.Z64, n, T.data_ptr(), n, ctypes.byref(o), info.data_ptr(), fl._stream_ptr())
    assert rc == 0
    W = _host(T)
    assert int(info.item()) == io == 0
    s = np.max(np.abs(Uo))
    for cols in (slice(0, 64), slice(n - 64, n)):
        assert np.max(np.abs(np.triu(W)[:, cols] - np.triu(Uo)[:, cols])) <= 1e-13 * s
    assert oracle.zfactor_backward_error(A, W) <= 1e-14


def test_complex_lookahead_leading_block():
    """n = 3072 at block 256: the outer loop's lookahead is on (more than 2048
    rows beyond the next block).  U's leading 512 x 512 block is the factor of
    A's leading block, against the oracle element by element; the whole
    factorization by its backward error."""
    n, k = 3072, 512
    A = inputs.hpd_bbh(n, 13)
    Uo, io = oracle.zpotrf(np.asfortranarray(A[:k, :k]))
    _, T = _dev(A, n)
    info = torch.zeros(1, dtype=torch.int32, device=DEV)
    o = fl.Opts(fl.VAR_RIGHT, 256, 0, 0, 0, 0)
    rc = fl.lib().flame_factor(fl.Z64, n, T.data_ptr(), n, ctypes.byref(o), info.data_ptr(), fl._stream_ptr())
    assert rc == 0
    W = _host(T)
    assert int(info.item()) == io == 0
    s = np.max(np.abs(Uo))
    assert np.max(np.abs(np.triu(W)[:k, :k] - np.triu(Uo))) <= 1e-13 * s
    assert oracle.zfactor_backward_error(A, W) <= 1e-14
