"""MI355X (gfx950) blocked Cholesky A = U^T U (arXiv 1601.05871,
Fig. "dense-chol" and its derived loop invariants).

Thin ctypes binding over ``libflame.so`` (declared in ``include/flame.h``):
argument marshalling only -- every step of the factorization, solve and
refinement runs in the library's HIP kernels.  PyTorch supplies device memory
and the current stream.  Importing this module does not load the library;
the first call does, and raises if it has not been built (there is no CPU
fallback).

Matrices are column-major: a 2-D torch tensor ``A`` with ``A.stride(0) == 1``
and ``A.stride(1) == lda >= n`` (for a contiguous row-major tensor pass
``A.mT``, or use :func:`colmajor`).  Only the upper triangle is read/written
(except by :func:`lu` and :func:`qr`, which factor general matrices, and
with ``lower=True``).
"""
from __future__ import annotations

import atexit
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libflame.so")

F64, F32, Z64 = 0, 1, 2
OPT_FIXED_NB = 1
OPT_LOWER = 2
VAR_AUTO, VAR_BORDERED, VAR_LEFT, VAR_RIGHT, VAR_BY_BLOCKS = 0, 1, 2, 3, 4
BY_BLOCKS_TILE = 128
TRAIL = {"native": 0, "f32": 1, "bf16": 2}
FLAME_OK, FLAME_ERR_HIP, FLAME_ERR_NOMEM, FLAME_ERR_NOT_CONVERGED, FLAME_ERR_UNSUPPORTED = 0, 1, 2, 3, 4
FLAME_ERR_BREAKDOWN = 5
REFINE = {"ir": 0, "cg": 1, "auto": 2}

SEL_FEATURES, SEL_HIDDEN, SEL_CLASSES = 5, 64, 12
SEL_NPARAM = 64 * 5 + 64 + 64 * 64 + 64 + 12 * 64 + 12

# every symbol include/flame.h declares
EXPORTS = (
    "flame_factor", "flame_solve", "flame_batched_factor", "flame_op_chol", "flame_op_trsm",
    "flame_op_gemm_tn", "flame_selector_load", "flame_select", "flame_select_logits", "flame_autotune",
    "flame_trace_enable", "flame_trace_collect", "flame_status_string", "flame_version",
    "flame_solve_mixed", "flame_shutdown", "flame_batched_factor_noalloc", "flame_trace_busy", "flame_probe",
    "flame_select_class", "flame_factor_by_blocks", "flame_by_blocks_tasks",
    "flame_ichol_analyze", "flame_ichol_stats", "flame_ichol_structure", "flame_ichol_factor", "flame_ichol_values",
    "flame_ichol_destroy", "flame_ichol_apply", "flame_ichol_pcg", "flame_lu", "flame_qr",
)
PROBE = {"mfma_f64": 0, "mfma_f32": 1, "mfma_bf16": 2, "copy": 3}
NOALLOC_MAX_BATCH = 262144
KC_CHOL, KC_TRSM, KC_GEMM, KC_OTHER = 0, 1, 2, 3


class FlameError(RuntimeError):
    def __init__(self, fn: str, status: int):
        self.status = status
        super().__init__(f"{fn} returned {status}: {status_string(status)}")


class Opts(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("nb", ctypes.c_int32), ("trail", ctypes.c_int32),
                ("lookahead", ctypes.c_int32), ("graph", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class Refine(ctypes.Structure):
    _fields_ = [("A0", ctypes.c_void_p), ("lda0", ctypes.c_int64), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("method", ctypes.c_int32)]


class SolveReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("method", ctypes.c_int32), ("eta_max", ctypes.c_double),
                ("shift", ctypes.c_double), ("factor_info", ctypes.c_int32), ("attempts", ctypes.c_int32)]


class IcholStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz_a", ctypes.c_int64), ("nnz_u", ctypes.c_int64), ("nbt", ctypes.c_int64),
                ("nblocks", ctypes.c_int64), ("ntasks", ctypes.c_int64), ("pool_bytes", ctypes.c_int64),
                ("flops", ctypes.c_double)]


class PcgOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


class PcgReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("relres", ctypes.c_double),
                ("bnorm", ctypes.c_double)]


class Choice(ctypes.Structure):
    _fields_ = [("cls", ctypes.c_int32), ("variant", ctypes.c_int32), ("nb", ctypes.c_int32),
                ("trail", ctypes.c_int32), ("flags", ctypes.c_int32), ("method", ctypes.c_int32),
                ("batched", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def _choice_dict(c: Choice) -> dict:
    return {"cls": c.cls, "variant": c.variant, "nb": c.nb,
            "trail": {v: k for k, v in TRAIL.items()}[c.trail], "fixed_nb": bool(c.flags & OPT_FIXED_NB),
            "method": {v: k for k, v in REFINE.items()}[c.method], "batched": bool(c.batched)}


class MixedOpts(ctypes.Structure):
    _fields_ = [("trail", ctypes.c_int32), ("nb", ctypes.c_int32), ("method", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double), ("scale", ctypes.c_int32),
                ("max_shifts", ctypes.c_int32), ("shift", ctypes.c_double), ("reserved", ctypes.c_int32),
                ("reserved2", ctypes.c_int32)]


_lib = None


def lib(path: str | None = None) -> ctypes.CDLL:
    """Loads libflame.so (built by ``python -m paper_1601_05871_amd.build``),
    or, on the first call, the library build at ``path`` (the sanitized one)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1601_05871_amd.build` "
                           "(the HIP library is required; there is no fallback)")
    L = ctypes.CDLL(path)
    i32, i64, vp, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_double
    L.flame_factor.argtypes = [i32, i64, vp, i64, ctypes.POINTER(Opts), vp, vp]
    L.flame_lu.argtypes = [i32, i64, vp, i64, vp, vp]
    L.flame_qr.argtypes = [i32, i64, i64, vp, i64, vp, vp, vp]
    L.flame_solve.argtypes = [i32, i64, i64, vp, i64, vp, i64, ctypes.POINTER(Refine),
                              ctypes.POINTER(SolveReport), vp]
    L.flame_batched_factor.argtypes = [i32, i32, vp, vp, vp, vp, ctypes.POINTER(Opts), vp]
    L.flame_op_chol.argtypes = [i32, i64, vp, i64, vp, i64, vp]
    L.flame_op_trsm.argtypes = [i32, i64, i64, vp, i64, vp, i64, vp]
    L.flame_op_gemm_tn.argtypes = [i32, i32, i32, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp]
    L.flame_selector_load.argtypes = [vp, i64]
    L.flame_select.argtypes = [i64, i64, i32, dbl, ctypes.POINTER(Choice)]
    L.flame_select_class.argtypes = [i32, ctypes.POINTER(Choice)]
    L.flame_select_logits.argtypes = [vp, i64, vp]
    L.flame_autotune.argtypes = [i32, i64, vp, i64, i64, i32, vp, vp]
    L.flame_trace_enable.argtypes = [i32]
    L.flame_trace_collect.argtypes = [vp, vp, vp, vp]
    L.flame_trace_busy.argtypes = [vp, vp]
    L.flame_probe.argtypes = [i32, i64, i32, vp, i64, i32, ctypes.POINTER(dbl), vp]
    L.flame_solve_mixed.argtypes = [i64, i64, vp, i64, vp, i64, vp, i64, ctypes.POINTER(MixedOpts),
                                    ctypes.POINTER(SolveReport), vp]
    L.flame_shutdown.argtypes = []
    L.flame_factor_by_blocks.argtypes = [i32, i64, vp, i64, vp, vp, vp]
    L.flame_by_blocks_tasks.argtypes = [i64, vp, vp, i64, ctypes.POINTER(i64)]
    L.flame_ichol_analyze.argtypes = [i64, vp, vp, i32, vp, vp, i64, i32, ctypes.POINTER(vp)]
    L.flame_ichol_stats.argtypes = [vp, ctypes.POINTER(IcholStats)]
    L.flame_ichol_structure.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.flame_ichol_factor.argtypes = [vp, vp, vp, vp]
    L.flame_ichol_values.argtypes = [vp, vp, vp]
    L.flame_ichol_destroy.argtypes = [vp]
    L.flame_ichol_apply.argtypes = [vp, vp, vp, vp]
    L.flame_ichol_pcg.argtypes = [vp, vp, vp, vp, ctypes.POINTER(PcgOpts), ctypes.POINTER(PcgReport), vp]
    L.flame_batched_factor_noalloc.argtypes = [i32, i32, vp, vp, vp, vp, vp]
    L.flame_status_string.argtypes = [ctypes.c_int]
    L.flame_status_string.restype = ctypes.c_char_p
    L.flame_version.argtypes = []
    L.flame_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("flame_status_string", "flame_version"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    # release graphs, streams and workspaces while the HIP runtime is still up
    # (atexit handlers run before the interpreter tears torch down)
    atexit.register(L.flame_shutdown)
    return L


def shutdown() -> None:
    """Waits for the devices and releases the library's cached graphs,
    streams, events and workspaces (re-created on the next call)."""
    _check("flame_shutdown", lib().flame_shutdown())


def status_string(status: int) -> str:
    return lib().flame_status_string(int(status)).decode()


def version() -> str:
    return lib().flame_version().decode()


def _check(fn: str, rc: int, ok=(FLAME_OK,)) -> int:
    if rc not in ok:
        raise FlameError(fn, rc)
    return rc


# ---- torch marshalling ------------------------------------------------------

def _torch():
    import torch
    return torch


def _stream_ptr() -> int:
    torch = _torch()
    return torch.cuda.current_stream().cuda_stream


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.complex128:
        return Z64  # flame_factor only
    raise TypeError(f"unsupported dtype {t.dtype} (float64, float32, or complex128 for factor)")


def _colmajor_ld(t, rows: int | None = None) -> int:
    """Leading dimension of a column-major 2-D device tensor."""
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    if not t.is_cuda:
        raise ValueError("expected a device (HIP) tensor")
    r, c = t.shape
    if c > 1 and r > 1 and t.stride(0) != 1:
        raise ValueError("expected column-major strides (1, lda); pass A.mT of a contiguous tensor")
    ld = t.stride(1) if c > 1 else max(r, 1)
    return max(int(ld), max(1, r))


def colmajor(t):
    """A column-major copy (or view) of a 2-D tensor with the same values."""
    return t.mT.contiguous().mT


def _opts(variant, nb, trail, lookahead, graph, fixed_nb=False) -> Opts:
    o = Opts()
    o.variant = int(variant)
    o.nb = int(nb)
    o.trail = TRAIL[trail] if isinstance(trail, str) else int(trail)
    o.lookahead = int(lookahead)
    o.graph = int(graph)
    o.flags = OPT_FIXED_NB if fixed_nb else 0
    return o


def factor(A, variant: int = VAR_RIGHT, nb: int = 128, trail="native", lookahead: int = 0, graph: int = 0,
           info=None, fixed_nb: bool = False, lower: bool = False):
    """A := Chol(A) in place (upper triangle; ``lower``: A = L L^T in the
    lower triangle, the upper one left as it is).  Returns the device int32
    ``info`` tensor (0, or the 1-based column of the first non-positive pivot).
    Asynchronous on the current stream.  ``fixed_nb``: the right-looking loop
    runs every block at ``nb`` (no smaller blocks in the last columns).
    complex128 A: the Hermitian factorization A = U^H U (A = L L^H with
    ``lower``), right-looking at native precision only."""
    torch = _torch()
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be a square 2-D tensor")
    n = A.shape[0]
    lda = _colmajor_ld(A)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    elif info.dtype != torch.int32 or info.numel() < 1 or not info.is_cuda:
        raise ValueError("info must be a device int32 tensor with at least one element")
    o = _opts(variant, nb, trail, lookahead, graph, fixed_nb)
    if lower:
        o.flags |= OPT_LOWER
    rc = lib().flame_factor(_dtype_code(A), n, A.data_ptr(), lda, ctypes.byref(o), info.data_ptr(), _stream_ptr())
    _check("flame_factor", rc)
    return info


def lu(A, info=None):
    """A := L\\U in place, LU without pivoting (flame_lu; FP64, column-major
    device tensor).  Returns the device int32 ``info`` (0, or the 1-based
    column of the first zero or non-finite pivot).  Asynchronous on the
    current stream."""
    torch = _torch()
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be a square 2-D tensor")
    if A.dtype != torch.float64:
        raise TypeError("flame_lu takes float64")
    n = A.shape[0]
    lda = _colmajor_ld(A)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    rc = lib().flame_lu(F64, n, A.data_ptr(), lda, info.data_ptr(), _stream_ptr())
    _check("flame_lu", rc)
    return info


def qr(A, tau=None, info=None):
    """A := the packed Householder QR of the m x n (m >= n) column-major FP64
    device tensor A in place (flame_qr): R in the upper triangle, the
    reflectors' vectors below the diagonal (LAPACK geqrf convention).
    Returns (tau, info): tau the n reflector scalars, info the device int32
    (0, or 1 if a wait between the panel kernel's workgroups gave up).
    Asynchronous on the current stream."""
    torch = _torch()
    if A.dim() != 2:
        raise ValueError("A must be a 2-D tensor")
    if A.dtype != torch.float64:
        raise TypeError("flame_qr takes float64")
    m, n = A.shape
    lda = _colmajor_ld(A)
    if tau is None:
        tau = torch.zeros(max(n, 1), dtype=torch.float64, device=A.device)
    elif tau.dtype != torch.float64 or tau.numel() < n or not tau.is_cuda:
        raise ValueError("tau must be a device float64 tensor with at least n elements")
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    rc = lib().flame_qr(F64, m, n, A.data_ptr(), lda, tau.data_ptr(), info.data_ptr(), _stream_ptr())
    _check("flame_qr", rc)
    return tau[:n], info


def _report(rep: SolveReport, rc: int) -> dict:
    return {"iters": rep.iters, "eta": rep.eta_max, "status": rc,
            "method": {v: k for k, v in REFINE.items()}.get(rep.method, rep.method),
            "shift": rep.shift, "factor_info": rep.factor_info, "attempts": rep.attempts}


def _square(name: str, t) -> int:
    if t.dim() != 2 or t.shape[0] != t.shape[1]:
        raise ValueError(f"{name} must be a square 2-D tensor")
    return int(t.shape[0])


def _rows(name: str, t, n: int) -> int:
    if t.dim() != 2 or t.shape[0] != n:
        raise ValueError(f"{name} must be a 2-D tensor with {n} rows")
    return int(t.shape[1])


def _pattern_bytes(pattern, nbt: int):
    import numpy as np

    if pattern is None:
        return None
    pat = np.ascontiguousarray(np.asarray(pattern, dtype=np.uint8))
    if pat.shape != (nbt, nbt):
        raise ValueError(f"pattern must be {nbt} x {nbt} (one entry per block of {BY_BLOCKS_TILE})")
    return pat


def factor_by_blocks(A, pattern=None, info=None):
    """Cholesky-by-blocks (flame_factor_by_blocks) in place on the FP64
    column-major A: 128 x 128 blocks as tasks of one persistent kernel;
    ``pattern`` (nbt x nbt, truthy = block (i, j) exists) gives the block
    incomplete factorization of that pattern, None the dense one.  Returns the
    device info tensor."""
    torch = _torch()
    n = _square("A", A)
    if A.dtype != torch.float64:
        raise TypeError("Cholesky-by-blocks takes float64 matrices")
    nbt = (n + BY_BLOCKS_TILE - 1) // BY_BLOCKS_TILE
    pat = _pattern_bytes(pattern, nbt)
    lda = _colmajor_ld(A)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    rc = lib().flame_factor_by_blocks(F64, n, A.data_ptr(), lda, None if pat is None else pat.ctypes.data,
                                      info.data_ptr(), _stream_ptr())
    _check("flame_factor_by_blocks", rc)
    return info


def by_blocks_tasks(nbt: int, pattern=None) -> list[tuple[int, int, int, int]]:
    """The task list of Cholesky-by-blocks for nbt x nbt blocks (host only):
    (type, k, i, j) with type 0 = CHOL(A_kk), 1 = TRSM(A_kj), 2 = update of
    A_ij from iteration k, in the order the kernel claims them."""
    import numpy as np

    pat = _pattern_bytes(pattern, int(nbt))
    pp = None if pat is None else pat.ctypes.data
    cnt = ctypes.c_int64(0)
    _check("flame_by_blocks_tasks", lib().flame_by_blocks_tasks(int(nbt), pp, None, 0, ctypes.byref(cnt)))
    out = np.zeros(4 * max(cnt.value, 1), dtype=np.int32)
    _check("flame_by_blocks_tasks", lib().flame_by_blocks_tasks(int(nbt), pp, out.ctypes.data, cnt.value,
                                                                 ctypes.byref(cnt)))
    return [tuple(int(x) for x in out[4 * q:4 * q + 4]) for q in range(cnt.value)]


def solve(U, B, A0=None, tol: float = 1e-13, max_iter: int = 30, method: str = "ir"):
    """Solves A X = B in place on B (column-major, n x nrhs) with A = U^T U.
    With ``A0`` (the original FP64 matrix) refines in FP64 with ``method``
    ('ir', 'cg' or 'auto', see flame.h) and returns the report (iters, eta,
    status, method); otherwise returns None.  Refinement synchronizes the
    stream."""
    torch = _torch()
    n = _square("U", U)
    nrhs = _rows("B", B, n)
    if B.dtype != U.dtype:
        raise TypeError("U and B must have the same dtype")
    if A0 is not None:
        _square("A0", A0)
        if A0.shape[0] != n:
            raise ValueError("A0 must be n x n")
        if A0.dtype != torch.float64 or U.dtype != torch.float64:
            raise TypeError("refinement needs float64 U, B and A0")
        if method not in REFINE:
            raise ValueError(f"method must be one of {sorted(REFINE)}")
    ldu = _colmajor_ld(U)
    ldb = _colmajor_ld(B)
    dt = _dtype_code(U)
    if A0 is None:
        rc = lib().flame_solve(dt, n, nrhs, U.data_ptr(), ldu, B.data_ptr(), ldb, None, None, _stream_ptr())
        _check("flame_solve", rc)
        return None
    ref = Refine()
    ref.A0 = A0.data_ptr()
    ref.lda0 = _colmajor_ld(A0)
    ref.tol = float(tol)
    ref.max_iter = int(max_iter)
    ref.method = REFINE[method]
    rep = SolveReport()
    rc = lib().flame_solve(dt, n, nrhs, U.data_ptr(), ldu, B.data_ptr(), ldb, ctypes.byref(ref), ctypes.byref(rep),
                           _stream_ptr())
    _check("flame_solve", rc, ok=(FLAME_OK, FLAME_ERR_NOT_CONVERGED))
    return _report(rep, rc)


def solve_mixed(A0, B, W=None, trail="bf16", nb: int = 0, tol: float = 1e-13, max_iter: int = 1000,
                method: str = "auto", scale: bool = True, max_shifts: int = 8, shift: float = 0.0):
    """Solves A0 X = B (in place on B) to FP64 backward error ``tol`` with a
    factor computed with ``trail`` trailing products (flame_solve_mixed):
    unit-diagonal scaling, shifted retries on breakdown, FP64 refinement.
    ``W`` (n x n float64, column-major) receives the factor; allocated when
    None.  Returns the report dict; raises on argument errors and on a
    breakdown of every attempt (FlameError with status FLAME_ERR_BREAKDOWN)."""
    torch = _torch()
    n = _square("A0", A0)
    nrhs = _rows("B", B, n)
    if A0.dtype != torch.float64 or B.dtype != torch.float64:
        raise TypeError("A0 and B must be float64")
    if W is None:
        W = torch.empty((n, n), dtype=torch.float64, device=A0.device).mT
    elif _square("W", W) != n or W.dtype != torch.float64:
        raise ValueError("W must be an n x n float64 tensor")
    if method not in REFINE:
        raise ValueError(f"method must be one of {sorted(REFINE)}")
    o = MixedOpts()
    o.trail = TRAIL[trail] if isinstance(trail, str) else int(trail)
    o.nb = int(nb)
    o.method = REFINE[method]
    o.max_iter = int(max_iter)
    o.tol = float(tol)
    o.scale = int(bool(scale))
    o.max_shifts = int(max_shifts)
    o.shift = float(shift)
    rep = SolveReport()
    rc = lib().flame_solve_mixed(n, nrhs, A0.data_ptr(), _colmajor_ld(A0), W.data_ptr(), _colmajor_ld(W),
                                 B.data_ptr(), _colmajor_ld(B), ctypes.byref(o), ctypes.byref(rep), _stream_ptr())
    _check("flame_solve_mixed", rc, ok=(FLAME_OK, FLAME_ERR_NOT_CONVERGED))
    out = _report(rep, rc)
    out["W"] = W
    return out


def batched_factor(ns, ptrs, ldas, info, dtype=F64, opts: Opts | None = None, graph: int | None = None):
    """Factors len(ns) matrices in one persistent launch.  ``ns``, ``ldas``,
    ``info``: device int32 tensors; ``ptrs``: device int64 tensor of matrix
    addresses.  ``graph``: 1 = capture / replay a HIP graph (the default), 0 =
    direct launch."""
    if graph is not None:
        opts = _opts(VAR_RIGHT, 0, 0, 0, graph)
    rc = lib().flame_batched_factor(int(dtype), int(ns.numel()), ns.data_ptr(), ptrs.data_ptr(), ldas.data_ptr(),
                                    info.data_ptr(), ctypes.byref(opts) if opts is not None else None,
                                    _stream_ptr())
    _check("flame_batched_factor", rc)
    return info


def batched_factor_noalloc(ns, ptrs, ldas, info, dtype=F64):
    """flame_batched_factor_noalloc: the batched factorization with its
    workspace in the library's fixed device array (no allocation; at most
    NOALLOC_MAX_BATCH matrices; overlapping calls on one GPU race)."""
    rc = lib().flame_batched_factor_noalloc(int(dtype), int(ns.numel()), ns.data_ptr(), ptrs.data_ptr(),
                                            ldas.data_ptr(), info.data_ptr(), _stream_ptr())
    _check("flame_batched_factor_noalloc", rc)
    return info


def batched_pointers(mats):
    """(ns, ptrs, ldas) device arrays for a list of square column-major device
    tensors of one dtype (marshalling for :func:`batched_factor`)."""
    torch = _torch()
    if not mats:
        raise ValueError("empty list")
    dev = mats[0].device
    ns = torch.tensor([int(M.shape[0]) for M in mats], dtype=torch.int32, device=dev)
    ptrs = torch.tensor([int(M.data_ptr()) for M in mats], dtype=torch.int64, device=dev)
    ldas = torch.tensor([_colmajor_ld(M) for M in mats], dtype=torch.int32, device=dev)
    return ns, ptrs, ldas


# ---- selector and autotuner ---------------------------------------------------

def selector_load(w) -> None:
    """Loads the selector MLP weights (float32, FLAME_SEL_NPARAM values in the
    header's order); ``None`` unloads them."""
    import numpy as np

    if w is None:
        _check("flame_selector_load", lib().flame_selector_load(None, 0))
        return
    w = np.ascontiguousarray(np.asarray(w, dtype=np.float32).reshape(-1))
    rc = lib().flame_selector_load(w.ctypes.data, int(w.size))
    _check("flame_selector_load", rc)


def select(n: int, batch: int = 1, dtype: int = F64, kappa: float = 0.0) -> dict:
    """The class the loaded selector ranks highest for this shape (runs its
    HIP kernel): a dict with the class number and its program."""
    c = Choice()
    rc = lib().flame_select(int(n), int(batch), int(dtype), float(kappa), ctypes.byref(c))
    _check("flame_select", rc)
    return _choice_dict(c)


def select_class(cls: int) -> dict:
    """The program of selector class ``cls``."""
    c = Choice()
    _check("flame_select_class", lib().flame_select_class(int(cls), ctypes.byref(c)))
    return _choice_dict(c)


def select_logits(features):
    """Class logits of the selector MLP for feature rows (count x 5, float32)."""
    import numpy as np

    f = np.ascontiguousarray(np.asarray(features, dtype=np.float32).reshape(-1, SEL_FEATURES))
    out = np.zeros((f.shape[0], SEL_CLASSES), dtype=np.float32)
    rc = lib().flame_select_logits(f.ctypes.data, int(f.shape[0]), out.ctypes.data)
    _check("flame_select_logits", rc)
    return out


def autotune(A, batch: int = 1, reps: int = 2):
    """Milliseconds per matrix of every selector class for solving A x = b
    (A left unchanged; +inf where a class cannot run or fails), 12 values in
    class order; records the fastest single-matrix factorization for
    VAR_AUTO.  ``batch``: the batch size the batched class is timed at."""
    import numpy as np

    n = _square("A", A)
    t = np.zeros(SEL_CLASSES, dtype=np.float64)
    rc = lib().flame_autotune(_dtype_code(A), n, A.data_ptr(), _colmajor_ld(A), int(batch), int(reps),
                              t.ctypes.data, _stream_ptr())
    _check("flame_autotune", rc)
    return t


def probe(kind: str, work: int, buf, reps: int = 3, wg_per_cu: int = 0) -> float:
    """Runs one measurement probe (flame_probe): TFLOP/s of an MFMA loop or
    GB/s of a device copy; ``buf`` is a device tensor used as scratch."""
    rate = ctypes.c_double(0.0)
    rc = lib().flame_probe(PROBE[kind], int(work), int(wg_per_cu), buf.data_ptr(), buf.numel() * buf.element_size(),
                           int(reps), ctypes.byref(rate), _stream_ptr())
    _check("flame_probe", rc)
    return rate.value


def trace_enable(on: bool = True) -> None:
    """Per-launch HIP-event timing of the library's kernels (instrumentation)."""
    _check("flame_trace_enable", lib().flame_trace_enable(int(bool(on))))


def trace_collect() -> dict:
    """Per kernel class: launches, ms (sum of launch durations), busy_ms (the
    union of the launches' intervals), flops, bytes; and span_ms, first start
    to last end (synchronizes)."""
    arr_i = (ctypes.c_int64 * 4)()
    ms, fl_, by = (ctypes.c_double * 4)(), (ctypes.c_double * 4)(), (ctypes.c_double * 4)()
    _check("flame_trace_collect", lib().flame_trace_collect(arr_i, ms, fl_, by))
    busy, span = (ctypes.c_double * 4)(), ctypes.c_double(0.0)
    _check("flame_trace_busy", lib().flame_trace_busy(busy, ctypes.byref(span)))
    names = ("chol", "trsm", "gemm", "other")
    out = {names[k]: {"launches": int(arr_i[k]), "ms": ms[k], "busy_ms": busy[k], "flops": fl_[k], "bytes": by[k]}
           for k in range(4)}
    out["span_ms"] = span.value
    return out


# ---- block operations of the loop body -------------------------------------

def op_chol(A, info, info_base: int = 0):
    rc = lib().flame_op_chol(_dtype_code(A), A.shape[0], A.data_ptr(), _colmajor_ld(A), info.data_ptr(),
                             int(info_base), _stream_ptr())
    _check("flame_op_chol", rc)


def op_trsm(U, X):
    b = _square("U", U)
    _rows("X", X, b)
    if X.dtype != U.dtype:
        raise TypeError("U and X must have the same dtype")
    rc = lib().flame_op_trsm(_dtype_code(U), X.shape[0], X.shape[1], U.data_ptr(), _colmajor_ld(U), X.data_ptr(),
                             _colmajor_ld(X), _stream_ptr())
    _check("flame_op_trsm", rc)


def op_gemm_tn(C, X, Y, upper: bool, trail="native", dtype=None):
    """C := C - X^T Y (upper triangle only if ``upper``).  For trail 'f32' /
    'bf16' X and Y are float32 / bfloat16 tensors and C is float64."""
    torch = _torch()
    if X.dim() != 2 or Y.dim() != 2 or C.dim() != 2:
        raise ValueError("C, X and Y must be 2-D tensors")
    k = X.shape[0]
    if Y.shape[0] != k:
        raise ValueError("X and Y must have the same number of rows (the inner dimension)")
    if C.shape[0] != X.shape[1] or C.shape[1] != Y.shape[1]:
        raise ValueError("C must be X.shape[1] x Y.shape[1]")
    if dtype is None:
        dtype = F32 if (C.dtype == torch.float32) else F64
    tr = TRAIL[trail] if isinstance(trail, str) else int(trail)
    rc = lib().flame_op_gemm_tn(int(dtype), tr, int(bool(upper)), C.shape[0], C.shape[1], k, X.data_ptr(),
                                _colmajor_ld(X), Y.data_ptr(), _colmajor_ld(Y), C.data_ptr(), _colmajor_ld(C),
                                _stream_ptr())
    _check("flame_op_gemm_tn", rc)


# ---- level(k) incomplete Cholesky by blocks (flame_ichol_*) --------------------

class IcholPlan:
    """A plan of the level(k) incomplete Cholesky-by-blocks (flame_ichol_*):
    the symbolic phase on construction (host CSR pattern ``rp`` / ``ci``, numpy
    int64 / int32), then ``factor(vals)`` with A's values on the device in the
    same entry order.  ``order`` / ``bounds``: optional ordering (new -> old)
    and block ranges; ``leaf``: leaf size of the library's dissection."""

    def __init__(self, n: int, rp, ci, level: int, order=None, bounds=None, leaf: int = 0):
        import numpy as np

        self._rp = np.ascontiguousarray(rp, dtype=np.int64)
        self._ci = np.ascontiguousarray(ci, dtype=np.int32)
        self._order = None if order is None else np.ascontiguousarray(order, dtype=np.int64)
        self._bounds = None if bounds is None else np.ascontiguousarray(bounds, dtype=np.int64)
        if self._rp.shape != (n + 1,):
            raise ValueError("rp must have n + 1 entries")
        if self._ci.shape != (int(self._rp[-1]),):
            raise ValueError("ci must have rp[n] entries")
        if self._order is not None and self._order.shape != (n,):
            raise ValueError("order must have n entries")
        self._h = ctypes.c_void_p()
        nr = 0 if self._bounds is None else len(self._bounds) - 1
        _check("flame_ichol_analyze", lib().flame_ichol_analyze(
            n, self._rp.ctypes.data, self._ci.ctypes.data, int(level),
            None if self._order is None else self._order.ctypes.data,
            None if self._bounds is None else self._bounds.ctypes.data, nr, int(leaf), ctypes.byref(self._h)))
        st = IcholStats()
        _check("flame_ichol_stats", lib().flame_ichol_stats(self._h, ctypes.byref(st)))
        self.stats = {f: getattr(st, f) for f, _ in IcholStats._fields_}
        self.n = n

    def structure(self) -> dict:
        """order, bounds, U's pattern (urp, uci, new numbering), the block
        pattern and the task list, as numpy arrays."""
        import numpy as np

        st = self.stats
        out = {"order": np.zeros(self.n, dtype=np.int64), "bounds": np.zeros(st["nbt"] + 1, dtype=np.int64),
               "urp": np.zeros(self.n + 1, dtype=np.int64), "uci": np.zeros(st["nnz_u"], dtype=np.int32),
               "pattern": np.zeros((st["nbt"], st["nbt"]), dtype=np.uint8),
               "tasks": np.zeros((st["ntasks"], 4), dtype=np.int32)}
        _check("flame_ichol_structure", lib().flame_ichol_structure(
            self._h, *[out[k].ctypes.data for k in ("order", "bounds", "urp", "uci", "pattern", "tasks")]))
        return out

    def factor(self, vals, info=None):
        """Numeric phase on the current stream; returns the device int32 info."""
        torch = _torch()
        if vals.dtype != torch.float64 or not vals.is_cuda or vals.numel() != self.stats["nnz_a"]:
            raise ValueError("vals must be a float64 device tensor with one value per entry of A")
        vals = vals.contiguous()
        if info is None:
            info = torch.zeros(1, dtype=torch.int32, device=vals.device)
        _check("flame_ichol_factor", lib().flame_ichol_factor(self._h, vals.data_ptr(), info.data_ptr(),
                                                              _stream_ptr()))
        return info

    def values(self):
        """U's values on its pattern (device float64, nnz_u)."""
        torch = _torch()
        out = torch.empty(self.stats["nnz_u"], dtype=torch.float64, device="cuda")
        _check("flame_ichol_values", lib().flame_ichol_values(self._h, out.data_ptr(), _stream_ptr()))
        return out

    def apply(self, r):
        """z = M^{-1} r with M = P^T U^T U P (device float64 n-vectors)."""
        torch = _torch()
        if r.dtype != torch.float64 or not r.is_cuda or r.numel() != self.n:
            raise ValueError("r must be a float64 device vector of n entries")
        r = r.contiguous()
        z = torch.empty_like(r)
        _check("flame_ichol_apply", lib().flame_ichol_apply(self._h, r.data_ptr(), z.data_ptr(), _stream_ptr()))
        return z

    def pcg(self, vals, b, x=None, tol: float = 1e-10, max_iter: int = 1000):
        """Preconditioned CG for A x = b (factor first); returns (x, report)
        with report = iters, status, relres, bnorm.  Synchronizes."""
        torch = _torch()
        for name, t in (("vals", vals), ("b", b)):
            if t.dtype != torch.float64 or not t.is_cuda:
                raise ValueError(f"{name} must be a float64 device tensor")
        if vals.numel() != self.stats["nnz_a"] or b.numel() != self.n:
            raise ValueError("vals must hold one value per entry of A and b n entries")
        vals, b = vals.contiguous(), b.contiguous()
        x = torch.zeros_like(b) if x is None else x
        if x.dtype != torch.float64 or not x.is_cuda or x.numel() != self.n or not x.is_contiguous():
            raise ValueError("x must be a contiguous float64 device vector of n entries")
        o = PcgOpts()
        o.tol, o.max_iter = float(tol), int(max_iter)
        rep = PcgReport()
        _check("flame_ichol_pcg", lib().flame_ichol_pcg(self._h, vals.data_ptr(), b.data_ptr(), x.data_ptr(),
                                                        ctypes.byref(o), ctypes.byref(rep), _stream_ptr()))
        return x, {"iters": rep.iters, "status": rep.status, "relres": rep.relres, "bnorm": rep.bnorm}

    def close(self) -> None:
        if self._h:
            lib().flame_ichol_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
