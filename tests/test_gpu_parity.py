"""GPU parity: the HIP path through the C ABI against the CPU oracle, on the
same seeded inputs.

Tolerances (FP64).  For A = B B^T + n I (kappa <~ 5) the oracle and the GPU
differ only by rounding order (MFMA reduction order, FMA contraction), so both
are within the backward-error bound gamma_{n+1} of the exact factor.  The test
bound for the factor is
  beta_F = ||A - U^T U||_F / ||A||_F <= 1e-14                       (target)
  max |U_gpu - U_oracle| / max |U_oracle| <= 1e-13                  (parity)
Exact-arithmetic input (scaled min(i, j)) must match bit for bit in every
precision.  FP32 factors: beta_F <= 2e-6, parity 1e-5.
"""
import numpy as np
import pytest
import torch

import inputs
import oracle
import paper_1601_05871_amd as fl
from gpu_util import to_dev, to_host, zeros_info

pytestmark = pytest.mark.gpu

TOL_BETA64 = 1e-14
TOL_PAR64 = 1e-13
TOL_BETA32 = 2e-6
TOL_PAR32 = 1e-5


def _rel_max(Ug, Uo):
    Ug, Uo = np.triu(Ug), np.triu(Uo)
    return float(np.max(np.abs(Ug - Uo)) / max(np.max(np.abs(Uo)), 1e-300)) if Uo.size else 0.0


# ---- block operations ---------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 5, 63, 64, 65, 100, 128, 129, 200, 255, 256])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_op_chol(n, dt):
    A = inputs.spd_bbt(n, n)
    Uo, io = oracle.potrf(A)
    Ad = to_dev(A, ld=n + 3, dtype=dt)
    info = zeros_info()
    fl.op_chol(Ad, info)
    Ug = to_host(Ad)
    assert int(info.item()) == io == 0
    tol = TOL_PAR64 if dt == torch.float64 else TOL_PAR32
    assert _rel_max(Ug, Uo) <= tol
    # strictly lower triangle untouched
    assert np.array_equal(np.tril(Ug, -1), np.tril(to_host(to_dev(A, dtype=dt)), -1))


@pytest.mark.parametrize("n", [1, 64, 100, 256])
def test_op_chol_minij_exact(n):
    A = inputs.minij_scaled(n)
    Ad = to_dev(A)
    info = zeros_info()
    fl.op_chol(Ad, info)
    assert int(info.item()) == 0
    assert np.array_equal(np.triu(to_host(Ad)), inputs.minij_factor(n))


@pytest.mark.parametrize("n,bad", [(10, 3), (64, 63), (100, 70), (256, 200)])
def test_op_chol_breakdown(n, bad):
    A = inputs.spd_bbt(n, 1)
    A[bad, bad] = -1.0
    _, io = oracle.potrf(A)
    Ad = to_dev(A)
    info = zeros_info()
    fl.op_chol(Ad, info, info_base=1000)
    assert io == bad + 1
    assert int(info.item()) == 1000 + bad + 1


@pytest.mark.parametrize("b,m", [(1, 1), (17, 63), (64, 130), (100, 65), (128, 200), (256, 129)])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_op_trsm(b, m, dt):
    g = np.random.Generator(np.random.PCG64(b * 1000 + m))
    U = np.asfortranarray(np.triu(g.standard_normal((b, b))) + 4.0 * np.eye(b))
    X = np.asfortranarray(g.standard_normal((b, m)))
    ref = oracle.trsm_upper_t(U, X)
    Ud = to_dev(U + np.tril(np.full((b, b), np.nan), -1), ld=b + 1, dtype=dt)  # lower = NaN: must not be read
    Xd = to_dev(X, ld=b + 2, dtype=dt)
    fl.op_trsm(Ud, Xd)
    got = to_host(Xd)
    tol = 1e-12 if dt == torch.float64 else 2e-4
    assert np.max(np.abs(got - ref)) <= tol * max(1.0, np.max(np.abs(ref)))


GEMM_SHAPES = [(1, 1, 1), (5, 7, 3), (130, 130, 17), (128, 128, 128), (300, 257, 64), (257, 300, 33), (64, 512, 256)]


@pytest.mark.parametrize("M,N,K", GEMM_SHAPES)
@pytest.mark.parametrize("upper", [False, True])
@pytest.mark.parametrize("padded", [False, True])
def test_op_gemm_f64(M, N, K, upper, padded):
    """With ``upper``, only C(i, j), i <= j, is updated (a trapezoid when
    M > N); everything below stays as it was."""
    g = np.random.Generator(np.random.PCG64(M * 7 + N * 3 + K))
    X = np.asfortranarray(g.standard_normal((K, M)))
    Y = np.asfortranarray(g.standard_normal((K, N)))
    C = np.asfortranarray(g.standard_normal((M, N)))
    if upper:
        ref = C.copy(order="F")
        full = oracle.gemm_tn(C, X, Y)
        iu = np.triu_indices(M, 0, N)
        ref[iu] = full[iu]
    else:
        ref = oracle.gemm_tn(C, X, Y)
    # odd leading dimensions exercise the unaligned (scalar-load) path
    pad = 1 if padded else 0
    Xd, Yd, Cd = to_dev(X, ld=K + pad), to_dev(Y, ld=K + pad), to_dev(C, ld=M + pad)
    fl.op_gemm_tn(Cd, Xd, Yd, upper)
    got = to_host(Cd)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, K)
    if upper:
        assert np.array_equal(np.tril(got, -1), np.tril(C, -1))


def test_op_gemm_f64_exact_structure():
    """Integer-valued operands: the MFMA product is exact, so any mistake in
    the operand/output lane layout (a transposed tile, a wrong k slot) shows
    as a bit difference."""
    M, N, K = 192, 160, 48
    g = np.random.Generator(np.random.PCG64(5))
    X = np.asfortranarray(g.integers(-8, 9, (K, M)).astype(np.float64))
    Y = np.asfortranarray(g.integers(-8, 9, (K, N)).astype(np.float64))
    C = np.asfortranarray(g.integers(-100, 101, (M, N)).astype(np.float64))
    ref = C - X.T @ Y
    Cd = to_dev(C)
    fl.op_gemm_tn(Cd, to_dev(X), to_dev(Y), False)
    assert np.array_equal(to_host(Cd), ref)


@pytest.mark.parametrize("trail", ["f32", "bf16"])
@pytest.mark.parametrize("M,N,K", [(130, 130, 64), (256, 384, 256), (17, 40, 16)])
def test_op_gemm_mixed(trail, M, N, K):
    """Low-precision operands, FP32 accumulation, FP64 C: compared with the
    oracle applied to the same rounded operands (the rounding is the caller's
    choice; the kernel must then be exact up to FP32 accumulation)."""
    g = np.random.Generator(np.random.PCG64(M + N + K))
    X = np.asfortranarray(g.standard_normal((K, M)))
    Y = np.asfortranarray(g.standard_normal((K, N)))
    C = np.asfortranarray(g.standard_normal((M, N)))
    lp = torch.float32 if trail == "f32" else torch.bfloat16
    Kp = (K + 15) // 16 * 16
    Xr = torch.zeros((Kp, M), dtype=lp)
    Yr = torch.zeros((Kp, N), dtype=lp)
    Xr[:K] = torch.from_numpy(X).to(lp)
    Yr[:K] = torch.from_numpy(Y).to(lp)
    ref = oracle.gemm_tn(C, np.asfortranarray(Xr.double().numpy()), np.asfortranarray(Yr.double().numpy()))
    Xd = Xr.T.contiguous().T.to("cuda:0")
    Yd = Yr.T.contiguous().T.to("cuda:0")
    Xd = Xd.as_strided(Xd.shape, (1, Kp))
    Yd = Yd.as_strided(Yd.shape, (1, Kp))
    Cd = to_dev(C)
    fl.op_gemm_tn(Cd, Xd, Yd, False, trail=trail, dtype=fl.F64)
    got = to_host(Cd)
    # FP32 accumulation of K products of magnitude <~ 1 (exact products)
    assert np.max(np.abs(got - ref)) <= 4 * K * 2.0 ** -24 * np.max(np.abs(Xr.double().numpy())) * \
        np.max(np.abs(Yr.double().numpy())) + 1e-12


# ---- full factorization -----------------------------------------------------

FACTOR_NS = [1, 2, 31, 100, 256, 513, 1000]


@pytest.mark.parametrize("variant", [1, 2, 3])
@pytest.mark.parametrize("nb", [32, 64, 128, 256])
@pytest.mark.parametrize("n", FACTOR_NS)
def test_factor_f64(variant, nb, n):
    A = inputs.spd_bbt(n, 0)
    Uo, io = oracle.potrf(A, threads=8)
    Ad = to_dev(A, ld=n + (n % 3))
    # fixed_nb: the right-looking loop runs the block size named here (without
    # it the last 6144 columns use blocks of at most 128)
    info = fl.factor(Ad, variant=variant, nb=nb, fixed_nb=True)
    Ug = to_host(Ad)
    assert int(info.item()) == io == 0
    assert _rel_max(Ug, Uo) <= TOL_PAR64
    assert oracle.factor_backward_error(A, Ug) <= TOL_BETA64
    assert np.array_equal(np.tril(Ug, -1), np.tril(to_host(to_dev(A, ld=n + (n % 3))), -1))


@pytest.mark.parametrize("n", [513, 1000, 1531])
@pytest.mark.parametrize("lookahead", [0, -1])
def test_factor_right_nb512_fixed(n, lookahead):
    """Blocks of 512 throughout (K = 512 trailing products, the 512-row CHOL
    and TRSM taken three levels deep), with and without lookahead."""
    A = inputs.spd_bbt(n, 21)
    Uo, _ = oracle.potrf(A, threads=8)
    Ad = to_dev(A, ld=n + 5)
    info = fl.factor(Ad, variant=3, nb=512, lookahead=lookahead, fixed_nb=True)
    Ug = to_host(Ad)
    assert int(info.item()) == 0
    assert _rel_max(Ug, Uo) <= TOL_PAR64
    assert oracle.factor_backward_error(A, Ug) <= TOL_BETA64


def test_factor_default_options_reach_schedule():
    """NULL options (variant chosen by the library, nb = 0) factor correctly;
    at this order the default schedule (512 / 256 / 128 by position) runs its
    128-column tail."""
    n = 1100
    A = inputs.spd_bbt(n, 22)
    Uo, _ = oracle.potrf(A, threads=8)
    Ad = to_dev(A)
    info = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    rc = fl.lib().flame_factor(fl.F64, n, Ad.data_ptr(), n, None, info.data_ptr(), fl._stream_ptr())
    assert rc == 0
    Ug = to_host(Ad)
    assert int(info.item()) == 0
    assert _rel_max(Ug, Uo) <= TOL_PAR64


@pytest.mark.parametrize("lookahead", [1, -1])
@pytest.mark.parametrize("nb", [64, 128])
def test_factor_right_lookahead_modes(lookahead, nb):
    n = 1531
    A = inputs.spd_bbt(n, 2)
    Uo, _ = oracle.potrf(A, threads=8)
    Ad = to_dev(A)
    info = fl.factor(Ad, variant=3, nb=nb, lookahead=lookahead)
    Ug = to_host(Ad)
    assert int(info.item()) == 0
    assert _rel_max(Ug, Uo) <= TOL_PAR64
    assert oracle.factor_backward_error(A, Ug) <= TOL_BETA64


@pytest.mark.parametrize("variant", [1, 2, 3])
@pytest.mark.parametrize("nb", [32, 128, 256])
def test_factor_minij_exact(variant, nb):
    n = 1000
    A = inputs.minij_scaled(n)
    Ad = to_dev(A)
    info = fl.factor(Ad, variant=variant, nb=nb)
    assert int(info.item()) == 0
    assert np.array_equal(np.triu(to_host(Ad)), inputs.minij_factor(n))


@pytest.mark.parametrize("variant", [1, 2, 3])
@pytest.mark.parametrize("nb", [64, 128])
def test_factor_f32(variant, nb):
    n = 700
    A = inputs.spd_bbt(n, 3)
    Uo, _ = oracle.potrf(A, threads=8)
    Ad = to_dev(A, dtype=torch.float32)
    info = fl.factor(Ad, variant=variant, nb=nb)
    Ug = to_host(Ad)
    assert int(info.item()) == 0
    assert _rel_max(Ug, Uo) <= TOL_PAR32
    assert oracle.factor_backward_error(A, Ug) <= TOL_BETA32


@pytest.mark.parametrize("variant", [1, 2, 3])
@pytest.mark.parametrize("bad", [0, 77, 500, 999])
def test_factor_breakdown_info(variant, bad):
    """A clearly indefinite pivot (diagonal entry -1 in a well-conditioned
    SPD matrix) must be reported at the same column by every variant."""
    n = 1000
    A = inputs.spd_bbt(n, 4)
    A[bad, bad] = -1.0
    _, io = oracle.potrf(A, threads=8)
    Ad = to_dev(A)
    info = fl.factor(Ad, variant=variant, nb=128)
    assert io == bad + 1
    assert int(info.item()) == bad + 1


def test_factor_after_breakdown_leaves_no_state():
    """Nothing a failed call leaves behind (its launches after the breakdown
    turn into no-ops on both streams of lookahead 2) may affect the next
    calls: an early breakdown, then two good factorizations of other orders,
    each equal to the oracle's factor."""
    A = inputs.spd_bbt(1500, 7)
    A[100, 100] = -1.0
    Ad = to_dev(A)
    assert int(fl.factor(Ad, variant=3, nb=128).item()) == 101
    for n, seed in ((1300, 8), (2100, 9)):
        A = inputs.spd_bbt(n, seed)
        Uo, io = oracle.potrf(A, threads=8)
        Ad = to_dev(A)
        info = fl.factor(Ad, variant=3, nb=128)
        Ug = to_host(Ad)
        assert int(info.item()) == io == 0
        assert _rel_max(Ug, Uo) <= TOL_PAR64
        assert oracle.factor_backward_error(A, Ug) <= TOL_BETA64


def test_factor_nan_info():
    n = 300
    A = inputs.spd_bbt(n, 5)
    A[150, 150] = np.nan
    Ad = to_dev(A)
    info = fl.factor(Ad, variant=3, nb=64)
    assert int(info.item()) == 151


def test_factor_zero_size():
    Ad = torch.zeros((0, 0), dtype=torch.float64, device="cuda:0")
    info = fl.factor(Ad, variant=3, nb=64)
    assert int(info.item()) == 0


def test_factor_deterministic():
    n = 1200
    A = inputs.spd_bbt(n, 6)
    outs = []
    for _ in range(2):
        Ad = to_dev(A)
        fl.factor(Ad, variant=3, nb=128)
        outs.append(to_host(Ad))
    assert np.array_equal(outs[0], outs[1])


def test_factor_graph_replays():
    n = 900
    A = inputs.spd_bbt(n, 7)
    Uo, _ = oracle.potrf(A, threads=8)
    Ad = to_dev(A)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for rep in range(3):
            Ad.copy_(to_dev(A))
            info = fl.factor(Ad, variant=3, nb=128, graph=1)
            s.synchronize()
            Ug = to_host(Ad)
            assert int(info.item()) == 0
            assert _rel_max(Ug, Uo) <= TOL_PAR64


_ORACLE_CACHE = {}


def _oracle_factor(n, seed):
    if (n, seed) not in _ORACLE_CACHE:
        A = inputs.spd_bbt(n, seed)
        _ORACLE_CACHE[(n, seed)] = (A, oracle.potrf(A, threads=8)[0])
    return _ORACLE_CACHE[(n, seed)]


@pytest.mark.parametrize("variant", [1, 2, 3])
@pytest.mark.parametrize("nb", [64, 256, 512])
def test_tall_k_products_split(variant, nb):
    """n = 2600: the left-looking and bordered loops' products with K up to
    ~2500 are split over K slices (partials added in slice order); nb = 512
    takes the diagonal factorization and the panel solve three levels deep."""
    n = 2600
    A, Uo = _oracle_factor(n, 12)
    Ad = to_dev(A, ld=n + 8)
    info = fl.factor(Ad, variant=variant, nb=nb, fixed_nb=True)
    assert int(info.item()) == 0
    Ug = to_host(Ad)
    assert _rel_max(Ug, Uo) <= TOL_PAR64
    assert oracle.factor_backward_error(A, Ug) <= TOL_BETA64


# ---- solve and refinement ------------------------------------------------------

# n spans single and multiple 128-row blocks with ragged tails; nrhs <= 8
# takes the single-launch FP64 path, larger nrhs the blocked one
@pytest.mark.parametrize("n,nrhs", [(1, 1), (100, 1), (127, 1), (128, 2), (129, 1), (513, 3), (1000, 8),
                                    (1000, 9), (1000, 64), (2500, 1)])
def test_solve_plain(n, nrhs):
    A = inputs.spd_bbt(n, 8)
    Uo, _ = oracle.potrf(A, threads=8)
    B = inputs.rhs(n, nrhs, 8)
    Xo = oracle.solve(np.triu(Uo), B)
    Ud = to_dev(A)
    fl.factor(Ud, variant=3, nb=128)
    Bd = to_dev(B, ld=n + 1)
    fl.solve(Ud, Bd)
    X = to_host(Bd)
    assert np.max(np.abs(X - Xo)) <= 1e-12 * max(1.0, np.max(np.abs(Xo)))
    assert oracle.solve_backward_error(A, X, B) <= 1e-14


def _forward_bound(A0, eta_gpu, eta_oracle):
    """Normwise forward-error bound of two solutions of A0 x = b with
    backward errors eta_gpu and eta_oracle: each is within
    2 eta kappa_inf / (1 - eta kappa_inf) of the exact x (perturbation theory
    for (A0 + dA) x = b + db, ||dA|| <= eta ||A0||, ||db|| <= eta ||b||)."""
    k_inf = np.linalg.norm(A0, np.inf) * np.linalg.norm(np.linalg.inv(A0), np.inf)
    one = lambda e: 2.0 * e * k_inf / max(1.0 - e * k_inf, 0.5)
    return one(eta_gpu) + one(eta_oracle)


@pytest.mark.parametrize("n,nrhs", [(100, 9), (128, 16), (129, 17), (700, 40), (1000, 64), (1281, 65),
                                    (2500, 130), (3000, 33)])
def test_solve_many_rhs(n, nrhs):
    """The matrix-core chain solves (more than 8 right-hand sides): ragged
    last row block, one to three 64-column launches, split sums; against the
    oracle's substitutions."""
    A = inputs.spd_bbt(n, 30)
    Uo, _ = oracle.potrf(A, threads=8)
    B = inputs.rhs(n, nrhs, 30)
    Xo = oracle.solve(np.triu(Uo), B)
    Ud = to_dev(A, ld=n + 3)
    assert int(fl.factor(Ud, variant=3, nb=128).item()) == 0
    Bd = to_dev(B, ld=n + 5)
    fl.solve(Ud, Bd)
    X = to_host(Bd)
    assert np.all(np.isfinite(X))
    assert np.max(np.abs(X - Xo)) <= 1e-12 * max(1.0, np.max(np.abs(Xo)))
    assert oracle.solve_backward_error(A, X, B) <= 1e-14


def test_solve_many_rhs_exact_structure():
    """min(i, j) factor U_ij = d_j and right-hand sides B = U^T U X for an
    integer X: both substitutions are exact in FP64 (every intermediate is an
    integer times a power of two), so X comes back bit for bit."""
    n, nrhs = 777, 20
    A = inputs.minij_scaled(n)
    U = inputs.minij_factor(n)
    g = np.random.Generator(np.random.PCG64(3))
    Xi = g.integers(-4, 5, size=(n, nrhs)).astype(np.float64)
    B = np.asfortranarray(U.T @ (U @ Xi))
    Ud = to_dev(A)
    assert int(fl.factor(Ud, variant=3, nb=128).item()) == 0
    Bd = to_dev(B)
    fl.solve(Ud, Bd)
    assert np.array_equal(to_host(Bd), Xi)


@pytest.mark.parametrize("trail", ["f32", "bf16"])
@pytest.mark.parametrize("kappa", [1e2, 1e4, 1e6])
@pytest.mark.parametrize("nrhs", [1, 64])
def test_mixed_factor_and_refinement(trail, kappa, nrhs):
    """flame_solve_mixed on A0 = Q diag(s) Q^T: unit-diagonal scaling, the
    low-precision factorization (shifted after a breakdown), FP64 refinement
    (IR while it halves eta, then preconditioned CG).  Every cell must reach
    eta <= 1e-13 (checked by the oracle's own metric), take at least one
    refinement step, and agree with the oracle's FP64 solution within the
    forward-error bound both backward errors imply."""
    n = 768
    A0 = inputs.spd_kappa(n, kappa, 0)
    B = inputs.rhs(n, nrhs, 0)
    Uo, io = oracle.potrf(A0, threads=8)
    assert io == 0
    x_star = oracle.solve(np.triu(Uo), B)
    A0d = to_dev(A0, ld=n + 2)
    Bd = to_dev(B, ld=n + 1)
    rep = fl.solve_mixed(A0d, Bd, trail=trail, nb=128, tol=1e-13, max_iter=2000, method="auto")
    X = to_host(Bd)
    assert rep["status"] == fl.FLAME_OK, rep
    assert rep["iters"] >= 1 and rep["factor_info"] == 0, rep
    # both etas at or below the target (near the rounding floor the two
    # residuals differ by their rounding order, so only the bound is compared;
    # test_refinement_eta_matches_oracle compares them where eta is large)
    eta = oracle.solve_backward_error(A0, X, B)
    assert eta <= 1e-13 and rep["eta"] <= 1e-13
    eta_o = oracle.solve_backward_error(A0, x_star, B)
    fwd = np.max(np.abs(X - x_star)) / np.max(np.abs(x_star))
    assert fwd <= _forward_bound(A0, eta, eta_o), (fwd, eta, eta_o)
    # A0 is not modified
    assert np.array_equal(np.triu(to_host(A0d)), np.triu(A0))


def test_mixed_bf16_high_kappa_needs_shift_and_cg():
    """kappa = 1e6 with BF16 products: the unshifted factorization breaks
    down on this input and classical refinement cannot converge
    (kappa u_bf16 >> 1), so the driver must have shifted and finished with
    CG."""
    n = 768
    A0 = inputs.spd_kappa(n, 1e6, 0)
    B = inputs.rhs(n, 1, 0)
    A0d = to_dev(A0)
    Bd = to_dev(B)
    rep = fl.solve_mixed(A0d, Bd, trail="bf16", nb=128, tol=1e-13, max_iter=2000, method="auto")
    assert rep["status"] == fl.FLAME_OK, rep
    assert rep["attempts"] >= 2 and rep["shift"] > 0.0, rep
    assert rep["method"] == "cg", rep
    assert oracle.solve_backward_error(A0, to_host(Bd), B) <= 1e-13


@pytest.mark.parametrize("method", ["ir", "cg"])
def test_mixed_methods_without_switch(method):
    """Each refinement method alone converges where it should: classical IR
    with FP32 products at kappa = 1e4, CG with BF16 products at kappa = 1e4."""
    n = 640
    trail = "f32" if method == "ir" else "bf16"
    A0 = inputs.spd_kappa(n, 1e4, 4)
    B = inputs.rhs(n, 3, 4)
    A0d = to_dev(A0)
    Bd = to_dev(B)
    rep = fl.solve_mixed(A0d, Bd, trail=trail, nb=128, tol=1e-13, max_iter=1000, method=method)
    assert rep["status"] == fl.FLAME_OK and rep["method"] == method, rep
    assert oracle.solve_backward_error(A0, to_host(Bd), B) <= 1e-13


def test_mixed_not_positive_diagonal_is_a_breakdown():
    n = 300
    A0 = inputs.spd_kappa(n, 1e2, 1)
    A0[40, 40] = -A0[40, 40]
    with pytest.raises(fl.FlameError) as e:
        fl.solve_mixed(to_dev(A0), to_dev(inputs.rhs(n, 1, 1)), trail="f32")
    assert e.value.status == fl.FLAME_ERR_BREAKDOWN


def test_mixed_every_attempt_breaks_down():
    """An indefinite matrix with a positive diagonal: no shift within the
    allowed retries makes it definite at BF16, so the driver reports a
    breakdown rather than a wrong factor."""
    n = 256
    g = np.random.Generator(np.random.PCG64(5))
    Q, _ = np.linalg.qr(g.standard_normal((n, n)))
    s = np.linspace(1.0, 2.0, n)
    s[-8:] = -1.0  # eight negative eigenvalues
    A0 = np.asfortranarray((Q * s) @ Q.T)
    A0 = np.asfortranarray(np.triu(A0) + np.triu(A0, 1).T)
    assert np.all(np.diag(A0) > 0)
    with pytest.raises(fl.FlameError) as e:
        fl.solve_mixed(to_dev(A0), to_dev(inputs.rhs(n, 1, 2)), trail="bf16", max_shifts=2)
    assert e.value.status == fl.FLAME_ERR_BREAKDOWN


def test_refinement_nrhs64_takes_correction_steps():
    """The blocked (nrhs > 8) refinement path: FP32-trailing factor, IR with
    at least one correction step, every column to eta <= 1e-13."""
    n = 900
    A0 = inputs.spd_kappa(n, 1e4, 6)
    B = inputs.rhs(n, 64, 6)
    Ad = to_dev(A0)
    A0d = to_dev(A0, ld=n + 3)
    assert int(fl.factor(Ad, variant=3, nb=128, trail="f32").item()) == 0
    Bd = to_dev(B, ld=n + 1)
    rep = fl.solve(Ad, Bd, A0=A0d, tol=1e-13, max_iter=30, method="ir")
    X = to_host(Bd)
    assert rep["status"] == fl.FLAME_OK and rep["iters"] >= 1, rep
    assert oracle.solve_backward_error(A0, X, B) <= 1e-13


@pytest.mark.parametrize("nrhs", [1, 9])
def test_refinement_cg_on_plain_factor(nrhs):
    """CG on the factor of flame_factor (BF16 products, kappa = 1e2): both the
    single-launch (nrhs <= 8) and the blocked (nrhs > 8) paths."""
    n = 700
    A0 = inputs.spd_kappa(n, 1e2, 7)
    B = inputs.rhs(n, nrhs, 7)
    Ad = to_dev(A0)
    A0d = to_dev(A0)
    assert int(fl.factor(Ad, variant=3, nb=128, trail="bf16").item()) == 0
    Bd = to_dev(B)
    rep = fl.solve(Ad, Bd, A0=A0d, tol=1e-13, max_iter=500, method="cg")
    assert rep["status"] == fl.FLAME_OK and rep["method"] == "cg" and rep["iters"] >= 1, rep
    assert oracle.solve_backward_error(A0, to_host(Bd), B) <= 1e-13


def test_mixed_graph_workspace_regrowth():
    """A graph captured for a mixed factorization at a small order must not be
    replayed into a panel workspace that a larger call has since replaced:
    capture at n = 600, grow the workspace with an eager n = 4096 call, then
    call the first configuration again and compare with the oracle."""
    n = 600
    A = inputs.spd_kappa(n, 1e2, 9)
    Uo, _ = oracle.potrf(A, threads=8)
    Ad = to_dev(A)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        info = fl.factor(Ad, variant=3, nb=128, trail="f32", graph=1)
        s.synchronize()
        first = to_host(Ad)
        big = to_dev(inputs.spd_bbt(4096, 9))
        assert int(fl.factor(big, variant=3, nb=256, trail="f32").item()) == 0
        torch.cuda.synchronize()
        del big
        filler = torch.full((1 << 24,), 7.0, dtype=torch.float64, device="cuda:0")  # reuse of freed memory
        Ad.copy_(to_dev(A))
        info = fl.factor(Ad, variant=3, nb=128, trail="f32", graph=1)
        s.synchronize()
        again = to_host(Ad)
        assert torch.all(filler == 7.0)
    assert int(info.item()) == 0
    assert np.array_equal(first, again)
    # FP32 products: the factor of a kappa = 1e2 matrix within FP32 rounding
    assert _rel_max(again, Uo) <= 1e-4


@pytest.mark.parametrize("nrhs", [1, 3, 9])
def test_refinement_eta_matches_oracle(nrhs):
    """With max_iter = 0 the reported eta is that of the first solve: checks
    the device residual and norms against the oracle's definition."""
    n = 700
    A0 = inputs.spd_kappa(n, 1e4, 3)
    B = inputs.rhs(n, nrhs, 3)
    Ad = to_dev(A0)
    A0d = to_dev(A0, ld=n + 3)
    fl.factor(Ad, variant=3, nb=128, trail="f32")
    Bd = to_dev(B, ld=n + 1)
    rep = fl.solve(Ad, Bd, A0=A0d, tol=0.0, max_iter=0)
    X = to_host(Bd)
    assert rep["iters"] == 0 and rep["status"] == fl.FLAME_ERR_NOT_CONVERGED
    eta_o = oracle.solve_backward_error(A0, X, B)
    assert eta_o > 1e-12  # the FP32-trailing factor leaves a visible residual
    assert abs(rep["eta"] - eta_o) <= 1e-3 * eta_o


def test_solve_refinement_converges_large():
    """Multi-block single-launch solves inside refinement (n = 3000)."""
    n = 3000
    A0 = inputs.spd_kappa(n, 1e3, 5)
    B = inputs.rhs(n, 1, 5)
    Ad = to_dev(A0)
    A0d = to_dev(A0)
    fl.factor(Ad, variant=3, nb=256, trail="f32")
    Bd = to_dev(B)
    rep = fl.solve(Ad, Bd, A0=A0d, tol=1e-14, max_iter=30)
    X = to_host(Bd)
    assert rep["status"] == fl.FLAME_OK and rep["iters"] >= 1, rep
    assert oracle.solve_backward_error(A0, X, B) <= 1.5e-14


def test_mixed_minij_exact():
    """The rounded panel of min(i, j) is exact in FP32 and BF16, so the mixed
    factor is exact too."""
    n = 600
    A = inputs.minij_scaled(n)
    for trail in ("f32", "bf16"):
        Ad = to_dev(A)
        info = fl.factor(Ad, variant=3, nb=128, trail=trail)
        assert int(info.item()) == 0
        assert np.array_equal(np.triu(to_host(Ad)), inputs.minij_factor(n))
