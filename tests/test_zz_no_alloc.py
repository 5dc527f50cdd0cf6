"""The no-allocation batched entry point (flame_batched_factor_noalloc)
against the allocating one (flame_batched_factor), through the C ABI: two
calls in a row on one GPU, the second with a smaller batch (its workspace
array keeps the first call's contents), each compared bit for bit with the
allocating path on the same inputs (the two share every kernel), and matrix
by matrix with the oracle."""
import ctypes

import numpy as np
import pytest
import torch

import inputs
import oracle
import paper_1601_05871_amd as fl

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _batch(seed, count, dtype, pad):
    """`count` SPD matrices with orders drawn from [1, 512] plus the edge
    orders 0 and 1024, one NaN-padded column-major buffer each."""
    g = np.random.Generator(np.random.PCG64(seed))
    ns = [int(x) for x in g.integers(1, 512, endpoint=True, size=count)] + [0, 1024]
    g.shuffle(ns)
    mats, bufs = [], []
    for i, n in enumerate(ns):
        A = inputs.spd_bbt(n, 500 + seed * 1000 + i) if n else np.zeros((0, 0))
        ld = max(1, n + pad)
        t = torch.full((max(n, 1) * ld,), float("nan"), dtype=dtype, device=DEV)
        if n:
            t.as_strided((n, n), (1, ld)).copy_(torch.from_numpy(A).to(dtype))
        mats.append(A)
        bufs.append((t, n, ld))
    return mats, bufs


def _arrays(bufs):
    ptrs = torch.tensor([b[0].data_ptr() for b in bufs], dtype=torch.int64, device=DEV)
    ldas = torch.tensor([b[2] for b in bufs], dtype=torch.int32, device=DEV)
    ns = torch.tensor([b[1] for b in bufs], dtype=torch.int32, device=DEV)
    return ns, ptrs, ldas


def _run(entry, bufs, code):
    ns, ptrs, ldas = _arrays(bufs)
    info = torch.full((len(bufs),), 99, dtype=torch.int32, device=DEV)
    stream = torch.cuda.current_stream().cuda_stream
    L = fl.lib()
    if entry == "noalloc":
        rc = L.flame_batched_factor_noalloc(code, len(bufs), ns.data_ptr(), ptrs.data_ptr(), ldas.data_ptr(),
                                            info.data_ptr(), stream)
    else:
        o = fl.Opts()
        o.graph = 0
        rc = L.flame_batched_factor(code, len(bufs), ns.data_ptr(), ptrs.data_ptr(), ldas.data_ptr(),
                                    info.data_ptr(), ctypes.byref(o), stream)
    assert rc == 0, rc
    torch.cuda.synchronize()
    return info.cpu().numpy()


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_noalloc_matches_allocating_entry_twice(dt):
    code = fl.F64 if dt == torch.float64 else fl.F32
    for call, (seed, count, pad) in enumerate([(1, 300, 2), (2, 60, 0)]):  # the second call is smaller
        print(f"[no_alloc] dtype={dt} call={call} batch={count + 2}", flush=True)
        mats, bufs_a = _batch(seed, count, dt, pad)
        _, bufs_b = _batch(seed, count, dt, pad)
        info_a = _run("alloc", bufs_a, code)
        info_b = _run("noalloc", bufs_b, code)
        assert np.array_equal(info_a, info_b)
        assert np.all(info_b == 0), info_b
        for A, (ta, n, ld), (tb, _, _) in zip(mats, bufs_a, bufs_b):
            # bit for bit with the allocating entry point (padding rows included)
            assert torch.equal(torch.nan_to_num(ta, nan=-7.0), torch.nan_to_num(tb, nan=-7.0)), n
            if n == 0:
                continue
            Ug = np.asfortranarray(tb.as_strided((n, n), (1, ld)).to("cpu", torch.float64).numpy())
            Uo, io = oracle.potrf(A, threads=8)
            assert io == 0
            rel = np.max(np.abs(np.triu(Ug) - np.triu(Uo))) / np.max(np.abs(Uo))
            assert rel <= (1e-13 if dt == torch.float64 else 1e-5), (n, rel)


def test_noalloc_rejects_a_batch_above_the_limit():
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the size check fails first
    rc = fl.lib().flame_batched_factor_noalloc(fl.F64, fl.NOALLOC_MAX_BATCH + 1, fake, fake, fake, fake, None)
    assert rc == -2
