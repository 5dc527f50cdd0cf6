"""Lower storage (FLAME_OPT_LOWER): A = L L^T with L in the lower triangle,
every variant, FP64 and FP32, ragged orders and padded leading dimensions,
against the oracle's upper factor transposed; the strictly upper triangle
(filled with markers) must come back bit for bit; breakdown columns."""
import numpy as np
import pytest
import torch

import inputs
import oracle
import paper_1601_05871_amd as fl

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _lower_input(A, ld, dtype):
    n = A.shape[0]
    g = np.random.Generator(np.random.PCG64(7))
    M = np.tril(A) + np.triu(g.standard_normal((n, n)) * 1e3 + 12345.0, 1)  # markers above the diagonal
    base = torch.full((max(n, 1) * ld,), float("nan"), dtype=dtype, device=DEV)
    T = base.as_strided((n, n), (1, ld))
    T.copy_(torch.from_numpy(M).to(dtype))
    return T, M


@pytest.mark.parametrize("variant,nb", [(fl.VAR_RIGHT, 64), (fl.VAR_LEFT, 128), (fl.VAR_BORDERED, 64),
                                        (fl.VAR_BY_BLOCKS, 0)])
@pytest.mark.parametrize("n", [1, 5, 64, 65, 127, 300, 1000])
def test_lower_f64(variant, nb, n):
    print(f"[lower] variant={variant} n={n}", flush=True)
    A = inputs.spd_bbt(n, 60)
    Uo, io = oracle.potrf(A, threads=8)
    T, M = _lower_input(A, n + 3, torch.float64)
    info = fl.factor(T, variant=variant, nb=nb, lower=True)
    W = T.cpu().numpy()
    assert int(info.item()) == io == 0
    L = np.tril(W)
    assert np.max(np.abs(L - np.triu(Uo).T)) <= 1e-13 * np.max(np.abs(Uo))
    iu = np.triu_indices(n, 1)
    assert np.array_equal(W[iu], M[iu])


def test_lower_f32_and_breakdown():
    n = 500
    A = inputs.spd_bbt(n, 61)
    Uo, _ = oracle.potrf(A, threads=8)
    T, M = _lower_input(A, n, torch.float32)
    assert int(fl.factor(T, variant=fl.VAR_RIGHT, nb=128, lower=True).item()) == 0
    W = T.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(np.tril(W) - np.triu(Uo).T)) <= 1e-5 * np.max(np.abs(Uo))
    iu = np.triu_indices(n, 1)
    assert np.array_equal(W[iu], M[iu].astype(np.float32).astype(np.float64))
    B = np.array(A, order="F", copy=True)
    B[222, 222] = -5.0
    T2, M2 = _lower_input(B, n, torch.float64)
    assert int(fl.factor(T2, variant=fl.VAR_RIGHT, nb=64, lower=True).item()) == oracle.potrf(B)[1] == 223
    W2 = T2.cpu().numpy()
    assert np.array_equal(W2[iu], M2[iu])


def test_lower_full_size_schedule():
    """n = 4096 in the default schedule (nb = 512 by position, lookahead 2)."""
    n = 4096
    A = inputs.spd_bbt(n, 62)
    Uo, _ = oracle.potrf(A, threads=16)
    T, M = _lower_input(A, n, torch.float64)
    assert int(fl.factor(T, variant=fl.VAR_RIGHT, nb=512, lookahead=2, lower=True).item()) == 0
    W = T.cpu().numpy()
    assert np.max(np.abs(np.tril(W) - np.triu(Uo).T)) <= 1e-13 * np.max(np.abs(Uo))
