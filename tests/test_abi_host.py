"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every symbol include/flame.h declares, argument validation returns
-i before anything touches the device, status strings, and the tile
enumeration of the trailing update (compiled for the host)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1601_05871_amd as fl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "flame.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(flame_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = fl.lib()
    declared = _declared()
    assert len(declared) >= 12
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(fl.EXPORTS) == declared


def test_version_and_status_strings():
    assert "gfx950" in fl.version()
    assert fl.status_string(0) == "success"
    assert "invalid" in fl.status_string(-3)
    assert "tolerance" in fl.status_string(fl.FLAME_ERR_NOT_CONVERGED)


def _opts(**kw):
    o = fl.Opts()
    for k, v in kw.items():
        setattr(o, k, v)
    return o


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


@pytest.mark.parametrize("args,expect", [
    ((7, 4, FAKE, 4, None, FAKE, None), -1),
    ((0, -1, FAKE, 4, None, FAKE, None), -2),
    ((0, 4, None, 4, None, FAKE, None), -3),
    ((0, 4, FAKE, 3, None, FAKE, None), -4),
    ((0, 4, FAKE, 4, None, None, None), -6),
])
def test_factor_argument_errors(args, expect):
    assert fl.lib().flame_factor(*args) == expect


@pytest.mark.parametrize("field,value", [("variant", 9), ("nb", 513), ("nb", -1), ("trail", 3),
                                         ("lookahead", 3), ("graph", 5), ])
def test_factor_bad_options(field, value):
    o = _opts(**{field: value})
    assert fl.lib().flame_factor(0, 4, FAKE, 4, ctypes.byref(o), FAKE, None) == -5


def test_factor_reserved_fields_must_be_zero():
    o = _opts()
    o.reserved[1] = 1
    assert fl.lib().flame_factor(0, 4, FAKE, 4, ctypes.byref(o), FAKE, None) == -5


def test_factor_unsupported_mixed_combinations():
    o = _opts(variant=3, trail=1)
    assert fl.lib().flame_factor(1, 4, FAKE, 4, ctypes.byref(o), FAKE, None) == fl.FLAME_ERR_UNSUPPORTED
    o = _opts(variant=2, trail=2)
    assert fl.lib().flame_factor(0, 4, FAKE, 4, ctypes.byref(o), FAKE, None) == fl.FLAME_ERR_UNSUPPORTED


def test_factor_complex_checks():
    """dtype FLAME_Z64 (complex): the right-looking loop at native precision
    only; option fields are checked as for the real dtypes, before any device
    call."""
    for kw in ({"variant": 1}, {"variant": 2}, {"variant": 4}, {"trail": 1}, {"trail": 2}):
        o = _opts(**kw)
        assert fl.lib().flame_factor(fl.Z64, 4, FAKE, 4, ctypes.byref(o), FAKE, None) == fl.FLAME_ERR_UNSUPPORTED
    for field, value in (("variant", 9), ("nb", 513), ("graph", 5), ("flags", 4)):
        o = _opts(**{field: value})
        assert fl.lib().flame_factor(fl.Z64, 4, FAKE, 4, ctypes.byref(o), FAKE, None) == -5
    assert fl.lib().flame_factor(fl.Z64, 4, FAKE, 3, None, FAKE, None) == -4
    assert fl.lib().flame_factor(3, 4, FAKE, 4, None, FAKE, None) == -1


def test_lu_argument_errors():
    L = fl.lib()
    assert L.flame_lu(7, 4, FAKE, 4, FAKE, None) == -1
    assert L.flame_lu(0, -1, FAKE, 4, FAKE, None) == -2
    assert L.flame_lu(0, 4, None, 4, FAKE, None) == -3
    assert L.flame_lu(0, 4, FAKE, 3, FAKE, None) == -4
    assert L.flame_lu(0, 4, FAKE, 4, None, None) == -5
    assert L.flame_lu(1, 4, FAKE, 4, FAKE, None) == fl.FLAME_ERR_UNSUPPORTED


def test_qr_argument_errors():
    L = fl.lib()
    assert L.flame_qr(7, 4, 4, FAKE, 4, FAKE, FAKE, None) == -1
    assert L.flame_qr(0, -1, 0, FAKE, 4, FAKE, FAKE, None) == -2
    assert L.flame_qr(0, 4, -1, FAKE, 4, FAKE, FAKE, None) == -3
    assert L.flame_qr(0, 4, 5, FAKE, 4, FAKE, FAKE, None) == -3  # n > m
    assert L.flame_qr(0, 4, 4, None, 4, FAKE, FAKE, None) == -4
    assert L.flame_qr(0, 4, 4, FAKE, 3, FAKE, FAKE, None) == -5
    assert L.flame_qr(0, 4, 4, FAKE, 4, None, FAKE, None) == -6
    assert L.flame_qr(0, 4, 4, FAKE, 4, FAKE, None, None) == -7
    assert L.flame_qr(1, 4, 4, FAKE, 4, FAKE, FAKE, None) == fl.FLAME_ERR_UNSUPPORTED
    assert L.flame_qr(0, 131073, 4, FAKE, 131073, FAKE, FAKE, None) == fl.FLAME_ERR_UNSUPPORTED


def test_solve_argument_errors():
    L = fl.lib()
    assert L.flame_solve(3, 4, 1, FAKE, 4, FAKE, 4, None, None, None) == -1
    assert L.flame_solve(0, -2, 1, FAKE, 4, FAKE, 4, None, None, None) == -2
    assert L.flame_solve(0, 4, -1, FAKE, 4, FAKE, 4, None, None, None) == -3
    assert L.flame_solve(0, 4, 1, None, 4, FAKE, 4, None, None, None) == -4
    assert L.flame_solve(0, 4, 1, FAKE, 2, FAKE, 4, None, None, None) == -5
    assert L.flame_solve(0, 4, 1, FAKE, 4, None, 4, None, None, None) == -6
    assert L.flame_solve(0, 4, 1, FAKE, 4, FAKE, 1, None, None, None) == -7
    r = fl.Refine()
    r.A0, r.lda0, r.tol, r.max_iter = None, 4, 1e-13, 3
    assert L.flame_solve(0, 4, 1, FAKE, 4, FAKE, 4, ctypes.byref(r), None, None) == -8
    r.A0 = 0x1000
    assert L.flame_solve(1, 4, 1, FAKE, 4, FAKE, 4, ctypes.byref(r), None, None) == fl.FLAME_ERR_UNSUPPORTED


def test_op_argument_errors():
    L = fl.lib()
    assert L.flame_op_chol(0, 257, FAKE, 300, FAKE, 0, None) == -2
    assert L.flame_op_trsm(0, 300, 4, FAKE, 300, FAKE, 300, None) == -2
    assert L.flame_op_gemm_tn(1, 2, 1, 4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 4, None) == -2
    assert L.flame_op_gemm_tn(0, 0, 1, 4, 4, 4, FAKE, 3, FAKE, 4, FAKE, 4, None) == -7
    assert L.flame_op_gemm_tn(0, 0, 1, 4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 3, None) == -11


def test_batched_and_selector_argument_errors():
    L = fl.lib()
    assert L.flame_batched_factor(2, 1, FAKE, FAKE, FAKE, FAKE, None, None) == -1
    assert L.flame_batched_factor(0, -1, FAKE, FAKE, FAKE, FAKE, None, None) == -2
    assert L.flame_selector_load(None, fl.SEL_NPARAM) == -1
    assert L.flame_selector_load(FAKE, 3) == -2
    ch = fl.Choice()
    assert L.flame_select(-1, 1, 0, 1.0, ctypes.byref(ch)) == -1
    assert L.flame_select(10, -1, 0, 1.0, ctypes.byref(ch)) == -2
    assert L.flame_select(10, 1, 5, 1.0, ctypes.byref(ch)) == -3
    assert L.flame_select(10, 1, 0, -1.0, ctypes.byref(ch)) == -4
    assert L.flame_select(10, 1, 0, 1.0, None) == -5
    assert L.flame_select_class(12, ctypes.byref(ch)) == -1
    o = _opts(variant=2)
    assert L.flame_batched_factor(0, 1, FAKE, FAKE, FAKE, FAKE, ctypes.byref(o), None) == -7
    assert L.flame_autotune(0, 4, FAKE, 4, 0, 1, FAKE, None) == -5
    assert L.flame_autotune(0, 4, FAKE, 4, 1, 0, FAKE, None) == -6
    assert L.flame_autotune(0, 4, FAKE, 4, 1, 1, None, None) == -7


TILE_PROBE = r'''
#include <cstdio>
#include <vector>
#include "tile_map.h"
using namespace flame;
int main() {
    for (int upper = 0; upper < 2; ++upper)
    for (int tm = 1; tm <= 40; ++tm)
    for (int tn = 1; tn <= 40; ++tn) {
        if (upper && tm > tn) continue;
        long long nt = tile_count(tm, tn, upper);
        long long expect = 0;
        for (int I = 0; I < tm; ++I) for (int J = 0; J < tn; ++J) if (!upper || I <= J) ++expect;
        if (nt != expect) { printf("count %d %d %d\n", upper, tm, tn); return 1; }
        std::vector<int> seen(tm * tn, 0);
        std::vector<int> seenw(nt, 0);
        for (long long w = 0; w < nt; ++w) {
            long long t = xcd_remap(w, nt);
            if (t < 0 || t >= nt || seenw[t]++) { printf("remap %lld\n", w); return 1; }
            int I, J; tile_of(t, tm, tn, upper, I, J);
            if (I < 0 || I >= tm || J < 0 || J >= tn || (upper && I > J) || seen[I * tn + J]++) {
                printf("tile %d %d %d t=%lld -> %d %d\n", upper, tm, tn, t, I, J); return 1; }
        }
    }
    printf("ok\n");
    return 0;
}
'''


def test_tile_enumeration_is_a_bijection(tmp_path):
    src = tmp_path / "probe.cpp"
    src.write_text(TILE_PROBE)
    exe = tmp_path / "probe"
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "paper_1601_05871_amd", "csrc"),
                    str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout


def test_factor_unknown_flag_bits():
    for bits in (4, 2 | 4, 1 << 30):  # 1 = FIXED_NB and 2 = LOWER are known
        o = _opts(flags=bits)
        assert fl.lib().flame_factor(0, 4, FAKE, 4, ctypes.byref(o), FAKE, None) == -5


def test_refine_method_must_be_known():
    r = fl.Refine()
    r.A0, r.lda0, r.tol, r.max_iter, r.method = 0x1000, 4, 1e-13, 3, 7
    assert fl.lib().flame_solve(0, 4, 1, FAKE, 4, FAKE, 4, ctypes.byref(r), None, None) == -8


def _mixed_opts(**kw):
    o = fl.MixedOpts()
    o.trail, o.method, o.max_iter, o.tol, o.scale, o.max_shifts = 2, 2, 10, 1e-13, 1, 4
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def test_solve_mixed_argument_errors():
    L = fl.lib()
    o = _mixed_opts()
    ok = ctypes.byref(o)
    assert L.flame_solve_mixed(-1, 1, FAKE, 4, FAKE, 4, FAKE, 4, ok, None, None) == -1
    assert L.flame_solve_mixed(4, -1, FAKE, 4, FAKE, 4, FAKE, 4, ok, None, None) == -2
    assert L.flame_solve_mixed(4, 1, None, 4, FAKE, 4, FAKE, 4, ok, None, None) == -3
    assert L.flame_solve_mixed(4, 1, FAKE, 3, FAKE, 4, FAKE, 4, ok, None, None) == -4
    assert L.flame_solve_mixed(4, 1, FAKE, 4, None, 4, FAKE, 4, ok, None, None) == -5
    assert L.flame_solve_mixed(4, 1, FAKE, 4, FAKE, 3, FAKE, 4, ok, None, None) == -6
    assert L.flame_solve_mixed(4, 1, FAKE, 4, FAKE, 4, None, 4, ok, None, None) == -7
    assert L.flame_solve_mixed(4, 1, FAKE, 4, FAKE, 4, FAKE, 3, ok, None, None) == -8
    assert L.flame_solve_mixed(4, 1, FAKE, 4, FAKE, 4, FAKE, 4, None, None, None) == -9
    for field, value in [("trail", 3), ("nb", 513), ("method", 3), ("max_iter", -1), ("tol", -1.0),
                         ("scale", 2), ("max_shifts", 65), ("shift", -1.0), ("reserved", 1)]:
        bad = _mixed_opts(**{field: value})
        assert L.flame_solve_mixed(4, 1, FAKE, 4, FAKE, 4, FAKE, 4, ctypes.byref(bad), None, None) == -9, field


def test_breakdown_status_string():
    assert "broke down" in fl.status_string(fl.FLAME_ERR_BREAKDOWN)


def test_shutdown_without_devices_is_a_no_op():
    assert fl.lib().flame_shutdown() == fl.FLAME_OK


# ---- the Python wrapper validates shapes before it touches the device --------

def test_wrapper_shape_checks():
    import torch

    z = torch.zeros
    with pytest.raises(ValueError):
        fl.solve(z(3, 4, dtype=torch.float64), z(3, 1, dtype=torch.float64))  # U not square
    with pytest.raises(ValueError):
        fl.solve(z(3, 3, dtype=torch.float64), z(4, 1, dtype=torch.float64))  # B rows != n
    with pytest.raises(TypeError):
        fl.solve(z(3, 3, dtype=torch.float64), z(3, 1, dtype=torch.float32))  # dtype mismatch
    with pytest.raises(ValueError):
        fl.solve(z(3, 3, dtype=torch.float64), z(3, 1, dtype=torch.float64), A0=z(4, 4, dtype=torch.float64))
    with pytest.raises(TypeError):
        fl.solve(z(3, 3, dtype=torch.float64), z(3, 1, dtype=torch.float64), A0=z(3, 3, dtype=torch.float32))
    with pytest.raises(ValueError):
        fl.solve(z(3, 3, dtype=torch.float64), z(3, 1, dtype=torch.float64), A0=z(3, 3, dtype=torch.float64),
                 method="gmres")
    with pytest.raises(ValueError):
        fl.op_trsm(z(3, 3), z(4, 2))  # X rows != b
    with pytest.raises(ValueError):
        fl.op_gemm_tn(z(4, 5), z(3, 4), z(2, 5), upper=False)  # inner dimensions differ
    with pytest.raises(ValueError):
        fl.op_gemm_tn(z(4, 4), z(3, 4), z(3, 5), upper=False)  # C not X.shape[1] x Y.shape[1]
    with pytest.raises(ValueError):
        fl.factor(z(3, 4, dtype=torch.float64))
    with pytest.raises(ValueError):
        fl.solve_mixed(z(3, 3, dtype=torch.float64), z(4, 1, dtype=torch.float64))
    with pytest.raises(TypeError):
        fl.solve_mixed(z(3, 3, dtype=torch.float32), z(3, 1, dtype=torch.float64))
