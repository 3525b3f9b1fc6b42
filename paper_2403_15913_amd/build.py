"""Build libkkt.so (HIP kernels for gfx950 + host C++) in-tree.

    python -m paper_2403_15913_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkkt.so")
ARCH = os.environ.get("KKT_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             # packed FP32 instructions stay disabled in all device code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall"]

SOURCES = [("kernels.hip", "hip"), ("api.cpp", "hip"), ("server.cpp", "hip"), ("noalloc.cpp", "hip"),
           ("ipm.cpp", "hip"), ("stagewise.cpp", "hip"),
           ("symbolic.cpp", "host")]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + r.stdout + r.stderr)


def build() -> str:
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    with tempfile.TemporaryDirectory() as tmp:
        objs = []
        for src, kind in SOURCES:
            path = os.path.join(CSRC, src)
            if not os.path.exists(path):
                continue
            obj = os.path.join(tmp, src + ".o")
            if kind == "hip":
                _run([hipcc, *HIP_FLAGS, "-x", "hip", "-c", path, "-o", obj])
            else:
                _run(["g++", *HOST_FLAGS, "-c", path, "-o", obj])
            objs.append(obj)
        out = os.path.join(tmp, "libkkt.so")
        _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", out])
        shutil.copyfile(out, LIB + ".tmp")
        os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build())
