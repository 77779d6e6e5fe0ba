"""Compile the oracle's C part (liboracle.so) with gcc.  Test infrastructure only."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "chebfd_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# -fcx-limited-range: textbook complex multiply (no inf/NaN recovery calls);
# no -ffast-math, so IEEE double rounding of each operation is kept.
CFLAGS = ["-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-fcx-limited-range"]


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
