"""Build the oracle's C part (TEST INFRASTRUCTURE ONLY).

``build_oracle()`` compiles ``sparse_ldl.c`` into ``_sparse_ldl.so`` next to
it with the host compiler; the tests and the CPU-baseline leg of the
benchmark load that library through ``oracle.sparse``.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sparse_ldl.c")
LIB = os.path.join(HERE, "_sparse_ldl.so")


def build_oracle(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O3", "-march=native", "-fPIC", "-shared", "-std=c99",
                    "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_oracle())
