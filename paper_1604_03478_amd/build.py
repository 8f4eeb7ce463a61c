"""Build of the HIP library liblbmmelt.so for gfx950 (in-tree)."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "liblbmmelt.so")
SOURCES = [os.path.join(CSRC, f) for f in
           ("lbm_kernels.hip", "lbm_adjoint.hip", "lbm_diag.hip", "lbm_front_heat.hip",
            "lbm_ceiling.hip", "lbm_capi.hip")]

# Packed FP32 instructions are disabled for every HIP translation unit.  Code
# object v5 keeps the library loadable by the HIP runtime that ships with the
# PyTorch wheel (the binding imports torch first, so both share one runtime).
HIPFLAGS = [
    "--offload-arch=gfx950", "-mcode-object-version=5", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast", "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    """Compile the library (always recompiles) and return its path."""
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *HIPFLAGS, "-I", INCLUDE, "-I", CSRC, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
