"""Build step of the HIP library: compiles csrc/ for gfx950 into
``libmhd355.so`` inside the package (in-tree, so that it travels with the
source tree).

FP64 arithmetic is compiled without FMA contraction: every kernel then
evaluates each formula in the written order, so results do not depend on the
tiling or launch shape.  Packed-FP32 instructions are disabled.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmhd355.so")
SOURCES = [os.path.join(CSRC, "mhd_lib.hip")]
DEPS = SOURCES + [os.path.join(CSRC, "mhd_kernels.hpp"),
                  os.path.join(os.path.dirname(HERE), "include", "mhd.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False, extra=None) -> str:
    cmd = [HIPCC] + FLAGS + list(extra or []) + ["-o", LIB + ".tmp"] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))
