"""Build the gfx950 shared library paper_2603_17481_amd/liblbm.so from csrc/.

hipcc cross-compiles for gfx950 without a GPU.  Packed FP32 instructions are
disabled for all device code (-packed-fp32-ops), and so is floating-point
contraction (the kernels' arithmetic is exactly the source's, in every kernel
that runs it).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "lbm.hip")
LIB = os.path.join(HERE, "liblbm.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-function",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = False, extra=None) -> str:
    cmd = [HIPCC] + FLAGS + list(extra or []) + [SRC, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=[a for a in sys.argv[1:] if a != "-v"]))
