"""Builds libsk.so (HIP for gfx950 + host C++) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsk.so")
SOURCES = ["sk_kernels.hip", "sk_rowshort.hip", "sk_fused.hip", "sk_runtime.hip", "sk_kpath.hip",
           "sk_static.hip", "sk_real.hip",
           "sk_solver.cpp", "sk_solver_real.cpp",
           "sk_serve.cpp", "sk_solve.cpp", "sk_newton.cpp", "sk_realhost.cpp"]
ARCH = os.environ.get("SK_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are kept out of the generated code.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    """Compiles every source and links libsk.so in the package directory."""
    out = LIB
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(bdir, src + ".o")
        if src.endswith(".hip"):
            cmd = ["hipcc", "-x", "hip", *HIP_FLAGS, "-c", path,
                   "-o", obj]
        else:
            cmd = ["hipcc", "-O3", "-std=c++17", "-fPIC", "-Wall", "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = out + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
