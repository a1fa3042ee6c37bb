"""Build step of the HIP library: compiles csrc/ for gfx950 into
``libmhd355.so`` inside the package (in-tree, so that it travels with the
source tree).

FP64 units are compiled with FMA contraction inside a statement
(-ffp-contract=on): every kernel evaluates each formula the same way
whatever the tiling or launch shape, so FP64 results are identical across
launch variants, and they agree with the oracle (plain C, no contraction,
IEEE division) to a few ulps per step.  The mixed path's FP32 kernels are
compiled in their own units with contraction across statements.
Packed-FP32 instructions are disabled.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmhd355.so")
# (source, extra flags): the FP64 kernels and the host runtime contract
# within a statement; the mixed path's FP32 kernels across statements.
UNITS = [
    (os.path.join(CSRC, "mhd_lib.hip"), ["-ffp-contract=on"]),
    (os.path.join(CSRC, "mhd_fp32.hip"), ["-ffp-contract=fast"]),
    (os.path.join(CSRC, "mhd_opt64.hip"), ["-ffp-contract=on"]),
    (os.path.join(CSRC, "mhd_opt32.hip"), ["-ffp-contract=fast"]),
]
SOURCES = [u[0] for u in UNITS]
DEPS = SOURCES + [os.path.join(CSRC, f) for f in ("mhd_kernels.hpp", "mhd_step.hpp")] + \
    [os.path.join(os.path.dirname(HERE), "include", "mhd.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False, extra=None) -> str:
    # the translation units compile concurrently
    objs, procs = [], []
    for src, fl in UNITS:
        obj = os.path.join(CSRC, os.path.basename(src) + ".o")
        cmd = [HIPCC] + FLAGS + fl + list(extra or []) + ["-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    for cmd, pr in procs:
        if pr.wait() != 0:
            raise subprocess.CalledProcessError(pr.returncode, cmd)
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    for o in objs:
        os.remove(o)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))
