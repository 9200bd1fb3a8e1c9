"""Build libfacert.so (renderer) and libfadenoise.so (denoiser), HIP for
gfx950, in the package directory."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "facert.hip")
LIB = os.path.join(HERE, "libfacert.so")
DN_SRC = os.path.join(HERE, "csrc", "denoise.hip")
DN_LIB = os.path.join(HERE, "libfadenoise.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # every fp32 operation of the decision arithmetic is rounded on its own
    "-ffp-contract=off",
    # packed-fp32 instructions stay off
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _compile(src: str, lib: str, verbose: bool) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *HIPCC_FLAGS, "-o", lib + ".tmp", src]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(lib + ".tmp", lib)
    return lib


def build(verbose: bool = False) -> str:
    _compile(DN_SRC, DN_LIB, verbose)
    return _compile(SRC, LIB, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
