"""The incomplete factorization's symbolic phase on the host (no GPU): the
library's level-k pattern (breadth-first fill paths) equals the oracle's
(symbolic elimination) on the same ordering; its task list is the by-blocks
list of its block pattern, every task after its dependences; its nested
dissection is a permutation that cuts the fill of the complete factor; the
flop count; argument validation."""
import ctypes

import numpy as np
import pytest

import inputs
import oracle.ichol as oi
import paper_1601_05871_amd as fl

from test_by_blocks_host import _check_order

CASES = [((16, 15), 5), ((13, 12), 9), ((7, 6, 6), 7), ((6, 5, 5), 27)]


def _oracle_bounds(ranges):
    return [0] + [e for _, e in ranges]


@pytest.mark.parametrize("dims,stencil", CASES)
@pytest.mark.parametrize("k", [0, 1, 2, 3])
@pytest.mark.parametrize("with_ranges", [True, False])
def test_pattern_equals_the_oracle(dims, stencil, k, with_ranges):
    rp, ci, v = inputs.laplacian_grid(dims, stencil)
    n = len(rp) - 1
    order, ranges = oi.nd_grid(dims, leaf=20)
    P = fl.IcholPlan(n, rp, ci, k, order=order, bounds=_oracle_bounds(ranges) if with_ranges else None)
    st = P.structure()
    urp, uci, _ = oi.permute_upper(n, rp, ci, v, order)
    orp, oci, _ = oi.fill_pattern(n, urp, uci, k)
    assert np.array_equal(st["urp"], orp) and np.array_equal(st["uci"], oci)
    assert np.array_equal(st["order"], order)
    b = st["bounds"]
    assert b[0] == 0 and b[-1] == n and np.all(np.diff(b) >= 1) and np.all(np.diff(b) <= 128)
    if with_ranges:  # the caller's ranges, cut into chunks of at most 128
        assert set(_oracle_bounds(ranges)) <= set(b.tolist())
    else:
        assert np.array_equal(b, np.r_[np.arange(0, n, 128), n])


@pytest.mark.parametrize("dims,stencil", CASES)
def test_block_pattern_and_task_list(dims, stencil):
    rp, ci, v = inputs.laplacian_grid(dims, stencil)
    n = len(rp) - 1
    order, ranges = oi.nd_grid(dims, leaf=12)
    P = fl.IcholPlan(n, rp, ci, 1, order=order, bounds=_oracle_bounds(ranges))
    st = P.structure()
    nbt = P.stats["nbt"]
    b = st["bounds"]
    blk = np.repeat(np.arange(nbt), np.diff(b))
    rows = np.repeat(np.arange(n), np.diff(st["urp"]))
    expect = np.zeros((nbt, nbt), dtype=np.uint8)
    expect[blk[rows], blk[st["uci"]]] = 1
    expect[np.arange(nbt), np.arange(nbt)] = 1
    assert np.array_equal(st["pattern"], expect)
    assert P.stats["nblocks"] == int(np.triu(expect).sum())
    tasks = [tuple(int(x) for x in t) for t in st["tasks"]]
    # the tasks of the block pattern (the by-blocks generators), each once, in a
    # claim order (a simulated list schedule) where every task follows the
    # tasks it waits for
    ref = fl.by_blocks_tasks(nbt, expect)
    assert len(tasks) == len(set(tasks)) == len(ref) and set(tasks) == set(ref)
    assert P.stats["ntasks"] == len(tasks)
    _check_order(tasks, lambda i, j: i == j or bool(expect[i][j]))
    # the updates of each block keep their iteration order
    seen = {}
    for ty, k, i, j in tasks:
        if ty == 2:
            assert seen.get((i, j), -1) < k
            seen[(i, j)] = k


def test_flop_count():
    rp, ci, v = inputs.laplacian_grid((9, 8))
    n = 72
    order, _ = oi.nd_grid((9, 8), leaf=10)
    P = fl.IcholPlan(n, rp, ci, 1, order=order)
    st = P.structure()
    pat = set()
    for i in range(n):
        for j in st["uci"][st["urp"][i]:st["urp"][i + 1]]:
            pat.add((i, int(j)))
    f = 0
    for k in range(n):
        row = [int(j) for j in st["uci"][st["urp"][k]:st["urp"][k + 1]]]
        f += len(row)
        for a, i in enumerate(row[1:], 1):
            for j in row[a:]:
                if (i, j) in pat:
                    f += 2
    assert P.stats["flops"] == f


@pytest.mark.parametrize("dims,stencil", [((48, 48), 5), ((14, 14, 14), 7)])
def test_library_dissection_cuts_the_fill(dims, stencil):
    """Nested dissection exists to cut fill: the complete factor's pattern
    with the library's ordering is well below the natural ordering's."""
    rp, ci, v = inputs.laplacian_grid(dims, stencil)
    n = len(rp) - 1
    P_nd = fl.IcholPlan(n, rp, ci, n, leaf=32)
    order = P_nd.structure()["order"]
    assert sorted(order.tolist()) == list(range(n))
    P_nat = fl.IcholPlan(n, rp, ci, n, order=np.arange(n))
    assert P_nd.stats["nnz_u"] < 0.6 * P_nat.stats["nnz_u"]


def test_disconnected_and_trivial_graphs():
    # two disjoint grids side by side, and a diagonal matrix
    rp1, ci1, _ = inputs.laplacian_grid((6, 6))
    n1 = 36
    rp = np.concatenate([rp1, rp1[1:] + rp1[-1]])
    ci = np.concatenate([ci1, ci1 + n1]).astype(np.int32)
    P = fl.IcholPlan(2 * n1, rp, ci, 2, leaf=8)
    assert sorted(P.structure()["order"].tolist()) == list(range(2 * n1))
    D = fl.IcholPlan(10, np.arange(11, dtype=np.int64), np.arange(10, dtype=np.int32), 3)
    assert D.stats["nnz_u"] == 10
    E = fl.IcholPlan(0, np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32), 1)
    assert E.stats["nbt"] == 0 and E.stats["ntasks"] == 0


def test_argument_errors():
    L = fl.lib()
    h = ctypes.c_void_p()
    rp = np.array([0, 1, 2], dtype=np.int64)
    ci = np.array([0, 1], dtype=np.int32)
    assert L.flame_ichol_analyze(-1, rp.ctypes.data, ci.ctypes.data, 0, None, None, 0, 0, ctypes.byref(h)) == -1
    assert L.flame_ichol_analyze(2, None, ci.ctypes.data, 0, None, None, 0, 0, ctypes.byref(h)) == -2
    assert L.flame_ichol_analyze(2, rp.ctypes.data, ci.ctypes.data, -1, None, None, 0, 0, ctypes.byref(h)) == -4
    bad = np.array([0, 5], dtype=np.int32)
    assert L.flame_ichol_analyze(2, rp.ctypes.data, bad.ctypes.data, 0, None, None, 0, 0, ctypes.byref(h)) == -3
    o = np.array([0, 0], dtype=np.int64)
    assert L.flame_ichol_analyze(2, rp.ctypes.data, ci.ctypes.data, 0, o.ctypes.data, None, 0, 0, ctypes.byref(h)) == -5
    o = np.array([1, 0], dtype=np.int64)
    bb = np.array([0, 3], dtype=np.int64)
    assert L.flame_ichol_analyze(2, rp.ctypes.data, ci.ctypes.data, 0, o.ctypes.data, bb.ctypes.data, 1, 0,
                                 ctypes.byref(h)) == -6
    assert L.flame_ichol_analyze(2, rp.ctypes.data, ci.ctypes.data, 0, None, bb.ctypes.data, 1, 0, ctypes.byref(h)) == -6
    assert L.flame_ichol_analyze(2, rp.ctypes.data, ci.ctypes.data, 0, None, None, 0, 0, None) == -9
    assert L.flame_ichol_stats(None, None) == -1
    assert L.flame_ichol_factor(None, None, None, None) == -1
    assert L.flame_ichol_destroy(None) == -1
