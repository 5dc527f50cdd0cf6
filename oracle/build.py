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


def build(src: str = SRC, out: str = LIB_PATH, extra: list[str] | None = None) -> str:
    cmd = ["gcc", *CFLAGS, *(extra or []), "-o", out + ".tmp", src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build())
