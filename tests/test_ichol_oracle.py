"""Pins of the oracle for the paper's own method, level(k) incomplete
Cholesky (oracle/ichol.py: O6 fill levels, O7 numeric factor), against what
fixes it independently: fill levels as shortest fill paths (Hysom and
Pothen's characterization, enumerated by brute force on small graphs),
the complete factorization (O1) when no fill is dropped, the closed-form
factor of the 1-D Laplacian, the defining property of the incomplete factor
((U^T U)_ij = A_ij on the pattern), the level-1 fill of the 5-point grid in
natural order, and the separator property of the grid ordering.  Mutants
planted in O6/O7 must each fail one of these."""
import os
from collections import deque

import numpy as np
import pytest

import inputs
import oracle
import oracle.ichol as oi
from oracle.build import SRC, build


def _natural_upper(rp, ci, val):
    n = len(rp) - 1
    return oi.permute_upper(n, rp, ci, val, np.arange(n))


def _dense_sym(n, rp, ci, val):
    D = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(rp))
    D[rows, ci] = val
    return D


def _path_levels(n, rp, ci, K):
    """Brute force: lev(i, j), i < j, = (length of the shortest path i .. j
    whose inner vertices are all < i) - 1, kept when <= K."""
    adj = [set(ci[rp[v]:rp[v + 1]].tolist()) - {v} for v in range(n)]
    out = {}
    for i in range(n):
        out[(i, i)] = 0
        dist = {i: 0}
        dq = deque([i])
        while dq:
            v = dq.popleft()
            if v != i and v > i:
                continue  # a vertex > i ends a path (it cannot be an inner vertex)
            for w in adj[v]:
                if w not in dist:
                    dist[w] = dist[v] + 1
                    if w < i:
                        dq.append(w)
                    elif w > i and dist[w] - 1 <= K:
                        out[(i, w)] = dist[w] - 1
        # only w > i reached through inner vertices < i count
    return out


def _random_graph(n, p, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    M = np.triu(g.uniform(size=(n, n)) < p, 1)
    M = M | M.T
    rows, cols = np.nonzero(M | np.eye(n, dtype=bool))
    o = np.lexsort((cols, rows))
    rows, cols = rows[o], cols[o]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp), cols.astype(np.int32), np.ones(len(cols))


@pytest.mark.parametrize("seed,n,p", [(1, 12, 0.2), (2, 25, 0.12), (3, 40, 0.06), (4, 30, 0.3)])
@pytest.mark.parametrize("K", [0, 1, 2, 3, 1000])
def test_levels_are_shortest_fill_paths(seed, n, p, K):
    rp, ci, v = _random_graph(n, p, seed)
    urp, uci, _ = _natural_upper(rp, ci, v)
    prp, pci, lev = oi.fill_pattern(n, urp, uci, K)
    got = {(i, int(j)): int(l) for i in range(n) for j, l in zip(pci[prp[i]:prp[i + 1]], lev[prp[i]:prp[i + 1]])}
    assert got == _path_levels(n, rp, ci, K)


def test_levels_on_an_ordered_grid_are_shortest_fill_paths():
    rp, ci, v = inputs.laplacian_grid((7, 6))
    order, _ = oi.nd_grid((7, 6), leaf=8)
    urp, uci, uv = oi.permute_upper(42, rp, ci, v, order)
    # the permuted full pattern for the brute force
    inv = np.empty(42, dtype=np.int64)
    inv[order] = np.arange(42)
    rows = inv[np.repeat(np.arange(42), np.diff(rp))]
    cols = inv[ci]
    o = np.lexsort((cols, rows))
    frp = np.zeros(43, dtype=np.int64)
    np.add.at(frp, rows[o] + 1, 1)
    frp = np.cumsum(frp)
    for K in (0, 1, 2, 4):
        prp, pci, lev = oi.fill_pattern(42, urp, uci, K)
        got = {(i, int(j)): int(l) for i in range(42) for j, l in zip(pci[prp[i]:prp[i + 1]], lev[prp[i]:prp[i + 1]])}
        assert got == _path_levels(42, frp, cols[o].astype(np.int32), K)


@pytest.mark.parametrize("dims,stencil", [((9, 8), 5), ((7, 7), 9), ((5, 4, 4), 7)])
def test_complete_pattern_gives_the_unblocked_factor(dims, stencil):
    """No fill dropped: O7's operations are O1's, so the factors agree bit for
    bit, and O1 is exactly zero off the pattern."""
    rp, ci, v = inputs.laplacian_grid(dims, stencil)
    n = len(rp) - 1
    order, _ = oi.nd_grid(dims, leaf=10)
    urp, uci, uv = oi.permute_upper(n, rp, ci, v, order)
    prp, pci, _ = oi.fill_pattern(n, urp, uci, n)
    U, info = oi.ichol(prp, pci, oi.values_on(prp, pci, urp, uci, uv))
    assert info == 0
    A = np.asfortranarray(oi.to_dense(urp, uci, uv))
    W, i1 = oracle.potrf(A)
    assert i1 == 0
    D = oi.to_dense(prp, pci, U)
    mask = oi.to_dense(prp, pci, np.ones(len(pci))) > 0
    assert np.array_equal(np.triu(W)[mask], D[mask])
    assert np.all(np.triu(W)[~mask & np.triu(np.ones((n, n), dtype=bool))] == 0.0)


def test_tridiagonal_level0_is_the_exact_factor():
    n = 50
    A = inputs.laplacian1d(n)
    rows, cols = np.nonzero(np.triu(A))
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp)
    ci = cols.astype(np.int32)
    val = np.triu(A)[rows, cols]
    prp, pci, _ = oi.fill_pattern(n, rp, ci, 0)
    assert np.array_equal(prp, rp) and np.array_equal(pci, ci)
    U, info = oi.ichol(prp, pci, oi.values_on(prp, pci, rp, ci, val))
    D = oi.to_dense(prp, pci, U)
    i = np.arange(n)
    # tridiag(-1, 2, -1) = U^T U with U_ii = sqrt((i+2)/(i+1)), U_i,i+1 = -sqrt((i+1)/(i+2))
    assert np.allclose(np.diag(D), np.sqrt((i + 2) / (i + 1)), rtol=1e-15, atol=0)
    assert np.allclose(np.diag(D, 1), -np.sqrt((i[:-1] + 1) / (i[:-1] + 2)), rtol=1e-15, atol=0)


@pytest.mark.parametrize("dims,stencil", [((12, 11), 5), ((10, 9), 9), ((6, 5, 5), 7), ((5, 5, 4), 27)])
@pytest.mark.parametrize("K", [0, 1, 2])
def test_incomplete_factor_matches_A_on_its_pattern(dims, stencil, K):
    rp, ci, v = inputs.laplacian_grid(dims, stencil)
    n = len(rp) - 1
    order, _ = oi.nd_grid(dims, leaf=12)
    urp, uci, uv = oi.permute_upper(n, rp, ci, v, order)
    prp, pci, _ = oi.fill_pattern(n, urp, uci, K)
    U, info = oi.ichol(prp, pci, oi.values_on(prp, pci, urp, uci, uv))
    assert info == 0
    D = oi.to_dense(prp, pci, U)
    A = oi.to_dense(urp, uci, uv)
    R = D.T @ D - (A + np.triu(A, 1).T)
    mask = oi.to_dense(prp, pci, np.ones(len(pci))) > 0
    assert np.max(np.abs(R[mask])) <= 1e-13 * np.max(np.abs(A))
    if K == 0:  # the dropped fill changes the factor
        Pc, Cc, _ = oi.fill_pattern(n, urp, uci, n)
        Uc, _ = oi.ichol(Pc, Cc, oi.values_on(Pc, Cc, urp, uci, uv))
        assert np.max(np.abs(oi.to_dense(Pc, Cc, Uc) - D)) > 1e-3


def test_level1_fill_of_the_natural_5_point_grid():
    """Natural order, m x m 5-point grid: eliminating p links its two higher
    neighbors p + 1 and p + m, so the level-1 fill is exactly the (m - 1)^2
    entries (p + 1, p + m), x < m - 1, y < m - 1."""
    m = 9
    rp, ci, v = inputs.laplacian_grid((m, m))
    urp, uci, _ = _natural_upper(rp, ci, v)
    prp, pci, lev = oi.fill_pattern(m * m, urp, uci, 1)
    fills = {(i, int(j)) for i in range(m * m) for j, l in zip(pci[prp[i]:prp[i + 1]], lev[prp[i]:prp[i + 1]]) if l == 1}
    expect = {(x + 1 + m * y, x + m * (y + 1)) for x in range(m - 1) for y in range(m - 1)}
    assert fills == expect


@pytest.mark.parametrize("dims", [(13, 9), (6, 7, 5), (16, 16)])
def test_grid_ordering_is_a_dissection(dims):
    """A valid permutation whose ranges tile [0, n); every edge between two
    ranges ends in a separator ordered after the other range (leaves touch
    only the separators of their ancestors, which come after them)."""
    rp, ci, v = inputs.laplacian_grid(dims, 9 if len(dims) == 2 else 27)
    n = len(rp) - 1
    order, ranges, is_sep = oi.nd_grid(dims, leaf=16, kinds=True)
    assert sorted(order.tolist()) == list(range(n))
    assert ranges[0][0] == 0 and ranges[-1][1] == n
    assert all(a[1] == b[0] for a, b in zip(ranges, ranges[1:]))
    assert is_sep[-1] and any(not s for s in is_sep)
    inv = np.empty(n, dtype=np.int64)
    inv[order] = np.arange(n)
    rng = np.empty(n, dtype=np.int64)
    for r, (s0, e0) in enumerate(ranges):
        rng[s0:e0] = r
    rows = np.repeat(np.arange(n), np.diff(rp))
    ra, rb = rng[inv[rows]], rng[inv[ci]]
    cross = ra != rb
    assert cross.any()
    later = np.maximum(ra[cross], rb[cross])
    assert all(is_sep[r] for r in later.tolist())


MUTANTS = {
    "levels_max_rule": ("const int64_t cand = (int64_t)lki + ulev[e] + 1;",
                        "const int64_t cand = (int64_t)(lki > ulev[e] ? lki : ulev[e]) + 1;"),
    "levels_no_increment": ("const int64_t cand = (int64_t)lki + ulev[e] + 1;",
                            "const int64_t cand = (int64_t)lki + ulev[e];"),
    "levels_skip_first_column": ("for (int64_t e = pos + 1; e < urp[k + 1]; ++e) { /* columns j > i of row k */",
                                 "for (int64_t e = pos + 2; e < urp[k + 1]; ++e) { /* columns j > i of row k */"),
    "ichol_update_sign": ("val[mid] = val[mid] - p;", "val[mid] = val[mid] + p;"),
    "ichol_skips_diagonal_target": ("for (int64_t qi = b + 1; qi <= qc; ++qi) {", "for (int64_t qi = b + 1; qi < qc; ++qi) {"),
    "ichol_unscaled_row": ("for (int64_t q = b + 1; q < e; ++q) val[q] = val[q] / piv;",
                           "for (int64_t q = b + 1; q < e; ++q) val[q] = val[q] / a;"),
}


def _ichol_pins_pass(L) -> bool:
    saved = oracle._lib
    oracle._lib = L
    try:
        checks = []
        rp, ci, v = _random_graph(25, 0.12, 2)
        urp, uci, _ = _natural_upper(rp, ci, v)
        for K in (1, 2):
            prp, pci, lev = oi.fill_pattern(25, urp, uci, K)
            got = {(i, int(j)): int(l) for i in range(25) for j, l in zip(pci[prp[i]:prp[i + 1]], lev[prp[i]:prp[i + 1]])}
            checks.append(got == _path_levels(25, rp, ci, K))
        rp, ci, v = inputs.laplacian_grid((9, 8))
        order, _ = oi.nd_grid((9, 8), leaf=10)
        urp, uci, uv = oi.permute_upper(72, rp, ci, v, order)
        prp, pci, _ = oi.fill_pattern(72, urp, uci, 1)
        U, info = oi.ichol(prp, pci, oi.values_on(prp, pci, urp, uci, uv))
        D = oi.to_dense(prp, pci, U)
        A = oi.to_dense(urp, uci, uv)
        mask = oi.to_dense(prp, pci, np.ones(len(pci))) > 0
        R = D.T @ D - (A + np.triu(A, 1).T)
        checks.append(info == 0 and np.max(np.abs(R[mask])) <= 1e-13 * np.max(np.abs(A)))
        return all(checks)
    finally:
        oracle._lib = saved


def test_real_oracle_passes_ichol_battery():
    assert _ichol_pins_pass(oracle.lib())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_ichol_mutant_fails_a_pin(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    mpath = os.path.join(tmp_path, f"oracle_{name}.c")
    with open(mpath, "w") as f:
        f.write(src.replace(old, new))
    lpath = build(mpath, os.path.join(tmp_path, f"liboracle_{name}.so"))
    assert not _ichol_pins_pass(oracle.load(lpath))


# ---- preconditioned conjugate gradients (the factor as a preconditioner) ----

def test_pcg_without_preconditioner_follows_scipy_cg():
    """M = I: the oracle's recurrences give scipy's CG iterates (same
    algorithm, independent code), iteration by iteration."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla

    rp, ci, v = inputs.laplacian_grid((14, 13))
    n = len(rp) - 1
    A = sp.csr_matrix((v, ci, rp), shape=(n, n))
    b = np.random.default_rng(3).standard_normal(n)
    for m in (1, 5, 20):
        x, it, _ = oi.pcg(rp, ci, v, b, tol=1e-300, max_iter=m)
        xs, _ = sla.cg(A, b, rtol=1e-300, atol=0.0, maxiter=m)
        assert it == m
        assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_pcg_with_complete_factor_takes_one_step():
    rp, ci, v = inputs.laplacian_grid((12, 11))
    n = len(rp) - 1
    order, _ = oi.nd_grid((12, 11), leaf=16)
    urp, uci, uv = oi.permute_upper(n, rp, ci, v, order)
    prp, pci, _ = oi.fill_pattern(n, urp, uci, n)
    U, _ = oi.ichol(prp, pci, oi.values_on(prp, pci, urp, uci, uv))
    b = np.random.default_rng(4).standard_normal(n)
    x, it, rel = oi.pcg(rp, ci, v, b, precond=lambda r: oi.triangular_apply(prp, pci, U, order, r), tol=1e-12)
    assert it == 1 and rel <= 1e-12


@pytest.mark.parametrize("dims,stencil", [((24, 22), 5), ((8, 8, 7), 7)])
def test_pcg_converges_and_higher_levels_help(dims, stencil):
    import scipy.sparse as sp

    rp, ci, v = inputs.laplacian_grid(dims, stencil)
    n = len(rp) - 1
    A = sp.csr_matrix((v, ci, rp), shape=(n, n))
    b = np.random.default_rng(5).standard_normal(n)
    order, _ = oi.nd_grid(dims, leaf=20)
    urp, uci, uv = oi.permute_upper(n, rp, ci, v, order)
    its = []
    for k in (None, 0, 1, 2):
        M = None
        if k is not None:
            prp, pci, _ = oi.fill_pattern(n, urp, uci, k)
            U, _ = oi.ichol(prp, pci, oi.values_on(prp, pci, urp, uci, uv))
            M = (lambda P, C, UU: (lambda r: oi.triangular_apply(P, C, UU, order, r)))(prp, pci, U)
        x, it, rel = oi.pcg(rp, ci, v, b, precond=M, tol=1e-10)
        assert rel <= 1e-10
        assert np.linalg.norm(b - A @ x) <= 1e-9 * np.linalg.norm(b)  # the true residual
        its.append(it)
    assert its[0] > its[1] >= its[2] >= its[3]
