"""Builds libflame.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

    python -m paper_1601_05871_amd.build              # libflame.so
    python -m paper_1601_05871_amd.build --sanitize   # libflame_san.so

The sanitized build instruments the host code only (AddressSanitizer and
UndefinedBehaviorSanitizer; every -fsanitize flag goes to the host pass
through -Xarch_host, the device code is built as usual); it is loaded by a
process that preloads clang's ASan runtime (tests/test_sanitize_host.py) and
serves the host-side checks of argument validation, task lists and the
selector's file parsing.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_PATH = os.path.join(HERE, "libflame.so")
BUILD_DIR = os.path.join(HERE, "_build")
LIB_SAN_PATH = os.path.join(HERE, "libflame_san.so")
BUILD_SAN_DIR = os.path.join(HERE, "_build_san")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _compile(src: str, build_dir: str = BUILD_DIR, extra: tuple = (), incremental: bool = False) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj):
        deps = [src, *glob.glob(os.path.join(CSRC, "*.h")), *glob.glob(os.path.join(INCLUDE, "*.h"))]
        if os.path.getmtime(obj) >= max(os.path.getmtime(d) for d in deps):
            return obj
    lang = ["-x", "hip"]
    cmd = [HIPCC, *FLAGS, *extra, *lang, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = False, sanitize: bool = False) -> str:
    """Compiles every source and links the library; returns its path.  With
    ``sanitize`` the host code is instrumented (libflame_san.so, objects kept
    in _build_san and recompiled only when a source or header changed)."""
    build_dir = BUILD_SAN_DIR if sanitize else BUILD_DIR
    out = LIB_SAN_PATH if sanitize else LIB_PATH
    extra = tuple(SAN_FLAGS) if sanitize else ()
    os.makedirs(build_dir, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda f: _compile(f, build_dir, extra, sanitize), srcs))
    tmp = out + ".tmp"
    # -z defs: a symbol left undefined (a kernel whose host stub the compiler
    # did not emit, say) fails the link here, not the load on the device host
    # (the sanitized library takes the sanitizer runtime as a dependency)
    link_extra = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-shared-libsan"] if sanitize else []
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,-z,defs", *link_extra, "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(out)
    return out


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
    sys.exit(0)
