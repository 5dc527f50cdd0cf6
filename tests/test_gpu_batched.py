"""Batched factorization (one persistent launch, orders sorted on the device)
against the oracle, matrix by matrix."""
import numpy as np
import pytest
import torch

import inputs
import oracle
import paper_1601_05871_amd as fl
from gpu_util import DEV

pytestmark = pytest.mark.gpu

EDGE_NS = [0, 1, 2, 15, 16, 17, 31, 32, 33, 47, 63, 64, 65, 100, 127, 128, 129, 255, 256, 257, 300, 511, 512, 513,
           777, 1024]


def _upload(mats, dtype, pad):
    """One device buffer per matrix (column-major, lda = n + pad, padding NaN)."""
    bufs = []
    for A in mats:
        n = A.shape[0]
        ld = max(1, n + pad)
        t = torch.full((max(n, 1) * ld,), float("nan"), dtype=dtype, device=DEV)
        if n:
            t.as_strided((n, n), (1, ld)).copy_(torch.from_numpy(A).to(dtype))
        bufs.append((t, n, ld))
    ptrs = torch.tensor([b[0].data_ptr() for b in bufs], dtype=torch.int64, device=DEV)
    ldas = torch.tensor([b[2] for b in bufs], dtype=torch.int32, device=DEV)
    ns = torch.tensor([b[1] for b in bufs], dtype=torch.int32, device=DEV)
    return bufs, ns, ptrs, ldas


def _download(buf):
    t, n, ld = buf
    torch.cuda.synchronize()
    return np.asfortranarray(t.as_strided((n, n), (1, ld)).to("cpu", torch.float64).numpy())


def _mats(seed, extra):
    g = np.random.Generator(np.random.PCG64(seed))
    ns = list(EDGE_NS) + [int(x) for x in g.integers(16, 512, endpoint=True, size=extra)]
    g.shuffle(ns)
    return [inputs._symmetrize_upper(inputs.spd_bbt(n, 100 + i)) if n else np.zeros((0, 0)) for i, n in
            enumerate(ns)]


@pytest.mark.parametrize("dt,pad", [(torch.float64, 0), (torch.float64, 3), (torch.float32, 1)])
def test_batched_matches_oracle(dt, pad):
    mats = _mats(1, 40)
    bufs, ns, ptrs, ldas = _upload(mats, dt, pad)
    info = torch.full((len(mats),), 99, dtype=torch.int32, device=DEV)
    fl.batched_factor(ns, ptrs, ldas, info, dtype=fl.F64 if dt == torch.float64 else fl.F32, graph=0)
    info_h = info.cpu().numpy()
    assert np.all(info_h == 0), info_h
    for A, buf in zip(mats, bufs):
        n = A.shape[0]
        if n == 0:
            continue
        Ug = _download(buf)
        Uo, io = oracle.potrf(A, threads=8)
        assert io == 0
        rel = np.max(np.abs(np.triu(Ug) - np.triu(Uo))) / np.max(np.abs(Uo))
        beta = oracle.factor_backward_error(A, Ug)
        if dt == torch.float64:
            assert rel <= 1e-13 and beta <= 1e-14, (n, rel, beta)
        else:
            assert rel <= 1e-5 and beta <= 2e-6, (n, rel, beta)
        # the strictly lower triangle and the padding rows are never written
        t, _, ld = buf
        full = t.to("cpu", torch.float64).numpy()
        M = full[: n * ld].reshape(n, ld).T  # rows of the padded column-major layout
        low = np.tril(np.ones((n, n), bool), -1)
        assert np.array_equal(M[:n][low], A.astype(np.float32 if dt == torch.float32 else np.float64)[low]
                              .astype(np.float64)), n
        if ld > n:
            assert np.all(np.isnan(M[n:])), n


def test_batched_breakdown_and_invalid_entries():
    """A clearly indefinite matrix reports the oracle's first bad pivot and
    leaves the others intact; bad sizes or leading dimensions get info = -1
    and their memory is not touched."""
    sizes = [40, 200, 33, 300, 64, 5]
    mats = [inputs.spd_bbt(n, 7 + i) for i, n in enumerate(sizes)]
    for k, j in ((1, 150), (3, 0), (4, 63)):
        mats[k][j, j] = -1e6 * sizes[k]
    bufs, ns, ptrs, ldas = _upload(mats, torch.float64, 0)
    ns_h = ns.cpu().numpy().copy()
    ld_h = ldas.cpu().numpy().copy()
    ns_h[5] = 1025       # order above the limit
    ld_h[2] = 32         # lda < n
    ns = torch.from_numpy(ns_h).to(DEV)
    ldas = torch.from_numpy(ld_h).to(DEV)
    info = torch.full((len(mats),), 99, dtype=torch.int32, device=DEV)
    fl.batched_factor(ns, ptrs, ldas, info, graph=0)
    info_h = info.cpu().numpy()
    for k, A in enumerate(mats):
        if k in (2, 5):
            assert info_h[k] == -1
            assert np.array_equal(_download(bufs[k]), A, equal_nan=True)
            continue
        Uo, io = oracle.potrf(A, threads=8)
        assert info_h[k] == io, (k, info_h[k], io)
        if io == 0:
            assert np.max(np.abs(np.triu(_download(bufs[k])) - np.triu(Uo))) <= 1e-13 * np.max(np.abs(Uo))


def test_batched_graph_replays_are_bitwise_equal():
    """The captured launch (replayed three times on fresh inputs) gives the
    same bytes as the direct launch; the sort order does not change results."""
    mats = _mats(2, 60)
    bufs, ns, ptrs, ldas = _upload(mats, torch.float64, 0)
    info = torch.zeros(len(mats), dtype=torch.int32, device=DEV)
    fl.batched_factor(ns, ptrs, ldas, info, graph=0)
    ref = [_download(b) for b in bufs]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for rep in range(3):
            for (t, n, ld), A in zip(bufs, mats):
                if n:
                    t.as_strided((n, n), (1, ld)).copy_(torch.from_numpy(A))
            info.fill_(99)
            fl.batched_factor(ns, ptrs, ldas, info, graph=1)
            s.synchronize()
            assert np.all(info.cpu().numpy() == 0)
            for b, R in zip(bufs, ref):
                assert np.array_equal(_download(b), R, equal_nan=True)


def test_batched_empty_and_all_tiny():
    info = torch.zeros(1, dtype=torch.int32, device=DEV)
    e = torch.zeros(0, dtype=torch.int32, device=DEV)
    fl.batched_factor(e, torch.zeros(0, dtype=torch.int64, device=DEV), e, info, graph=0)
    mats = [np.array([[4.0]]), np.array([[9.0, 3.0], [3.0, 5.0]])] * 50
    bufs, ns, ptrs, ldas = _upload(mats, torch.float64, 0)
    info = torch.full((len(mats),), 99, dtype=torch.int32, device=DEV)
    fl.batched_factor(ns, ptrs, ldas, info)
    assert np.all(info.cpu().numpy() == 0)
    for A, b in zip(mats, bufs):
        U = np.triu(_download(b))
        exp = np.array([[2.0]]) if A.shape[0] == 1 else np.array([[3.0, 1.0], [0.0, 2.0]])
        assert np.array_equal(U, exp)


def test_batched_workload_sample():
    """The benchmark's workload (n ~ U{16..512}, 10,000 matrices, FP64),
    checked on a sample of matrices: every info is 0 and each sampled factor
    is within the parity bound of the oracle."""
    count = 10000
    sizes, mats = inputs.batch_torch(count, 0, DEV)
    pristine = {i: mats[i].cpu().numpy() for i in range(0, count, 331)}
    ns, ptrs, ldas = fl.batched_pointers(mats)
    info = torch.full((count,), 99, dtype=torch.int32, device=DEV)
    fl.batched_factor(ns, ptrs, ldas, info)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    for i, A in pristine.items():
        Ug = np.asfortranarray(mats[i].cpu().numpy())
        Uo, io = oracle.potrf(np.asfortranarray(A), threads=8)
        assert io == 0
        assert np.max(np.abs(np.triu(Ug) - np.triu(Uo))) <= 1e-13 * np.max(np.abs(Uo)), (i, sizes[i])
