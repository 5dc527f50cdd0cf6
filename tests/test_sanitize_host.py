"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

The oracle (gcc build, liboracle_san.so) runs its factor, blocked variants,
block operations, solve and by-blocks loop on small inputs and must give the
plain build's results bit for bit; the library's host code (hipcc build with
-Xarch_host sanitizers, libflame_san.so) runs its argument validation, the
by-blocks task lists, the selector's weight parsing and class table, and
shutdown.  Each runs in a child process that preloads its compiler's ASan
runtime; any sanitizer report fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run_preloaded(runtime: str, code: str):
    env = dict(os.environ)
    env["LD_PRELOAD"] = runtime
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1:exitcode=23"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=24"
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT,
                       timeout=600)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-4000:]
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    assert "sanitized-ok" in r.stdout, report[-4000:]


def _gcc_asan() -> str:
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(p) or not os.path.exists(p):
        pytest.skip("gcc's libasan is not installed")
    return p


def _clang_asan() -> str:
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        pytest.skip("clang's ASan runtime is not installed")
    return hits[-1]


ORACLE_CODE = r'''
import numpy as np
import inputs, oracle
from oracle import build as ob
plain = oracle.load(ob.LIB_PATH if __import__("os").path.exists(ob.LIB_PATH) else ob.build())
san = oracle.load(ob.build(sanitize=True))
def run(L):
    oracle._lib = L
    out = []
    for n in (1, 7, 64, 150):
        A = inputs.spd_bbt(n, 3)
        out.append(oracle.potrf(A, threads=2)[0])
        for v in (1, 2, 3):
            out.append(oracle.potrf_blocked(A, b=16, variant=v)[0])
        out.append(oracle.chol_by_blocks(A, None, b=32)[0])
        U = out[-1]
        B = inputs.rhs(n, 2, 4)
        out.append(oracle.solve(U, B))
    X = np.asfortranarray(np.random.default_rng(1).standard_normal((40, 30)))
    out.append(oracle.trsm_upper_t(np.triu(inputs.spd_bbt(40, 5)) + 40 * np.eye(40), X))
    out.append(oracle.syrk_upper(X, np.asfortranarray(np.zeros((30, 30)))))
    return out
ctypes = __import__("ctypes")
ctypes.CDLL(None).__asan_init  # the preloaded runtime is there
a, b = run(plain), run(san)
assert all(np.array_equal(x, y) for x, y in zip(a, b))
print("sanitized-ok")
'''


def test_oracle_under_sanitizers():
    rt = _gcc_asan()
    _run_preloaded(rt, ORACLE_CODE)


LIB_CODE = r'''
import ctypes, json, os
import numpy as np
from paper_1601_05871_amd import build as lb
import paper_1601_05871_amd as fl
L = fl.lib(lb.build(sanitize=True))
ctypes.CDLL(None).__asan_init  # the preloaded runtime is there
FAKE = ctypes.c_void_p(0x1000)
assert L.flame_factor(7, 4, FAKE, 4, None, FAKE, None) == -1
assert L.flame_factor(0, 4, FAKE, 3, None, FAKE, None) == -4
o = fl.Opts(); o.nb = 513
assert L.flame_factor(0, 4, FAKE, 4, ctypes.byref(o), FAKE, None) < 0
for code in (0, -3, fl.FLAME_ERR_NOT_CONVERGED, 5, 12345):
    assert isinstance(fl.status_string(code), str)
assert "gfx950" in fl.version()
# by-blocks task lists: dense and with patterns, sizes up to 40 blocks
for nbt in (0, 1, 2, 5, 17, 40):
    t = fl.by_blocks_tasks(nbt)
    P = (np.random.default_rng(nbt).uniform(size=(nbt, nbt)) < 0.3).astype(np.uint8)
    t2 = fl.by_blocks_tasks(nbt, P)
    assert len(t2) <= len(t)
# selector weights: a full parameter vector, then wrong counts, then unload
w = np.random.default_rng(0).standard_normal(fl.SEL_NPARAM).astype(np.float32)
assert L.flame_selector_load(w.ctypes.data, w.size) == 0
assert L.flame_selector_load(w.ctypes.data, w.size - 1) == -2
assert L.flame_selector_load(None, 5) == -1
assert L.flame_selector_load(None, 0) == 0
ch = fl.Choice()
for c in range(-1, 14):
    L.flame_select_class(c, ctypes.byref(ch))
fl.shutdown()
print("sanitized-ok")
'''


def test_library_host_code_under_sanitizers():
    rt = _clang_asan()
    _run_preloaded(rt, LIB_CODE)
