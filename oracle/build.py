"""Builds liboracle.so from oracle.c with the host C compiler (test
infrastructure; see the package docstring)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB_PATH = os.path.join(HERE, "liboracle.so")

# IEEE binary64, no FMA contraction, no fast-math: every operation is the one
# the source writes.
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11"]
# AddressSanitizer + UndefinedBehaviorSanitizer build (liboracle_san.so), for a
# process that preloads gcc's libasan (tests/test_sanitize_host.py); the same
# floating-point flags, so its results are the plain build's bit for bit.
SAN_PATH = os.path.join(HERE, "liboracle_san.so")
SAN_FLAGS = ["-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def build(src: str = SRC, out: str = LIB_PATH, extra: list[str] | None = None, sanitize: bool = False) -> str:
    if sanitize:
        extra = [*SAN_FLAGS, *(extra or [])]
        out = SAN_PATH if out == LIB_PATH else out
    cmd = ["gcc", *CFLAGS, *(extra or []), "-o", out + ".tmp", src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build())
