"""Build step of the CPU oracle (test infrastructure only).

Compiles ``mhd_oracle.c`` with gcc into ``liboracle.so`` next to this file.
FP64, no fused multiply-add contraction, IEEE division and square root.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mhd_oracle.c")
# A test may point the wrapper at a deliberately mutated build of the oracle
# (tests/test_oracle_mutations.py) through MHD_ORACLE_LIB.
LIB = os.environ.get("MHD_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")


def compile_to(src: str, lib: str, verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O3", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared",
        "-ffp-contract=off", "-fno-fast-math", "-I", HERE,
        "-o", lib + ".tmp", src, "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


def build(verbose: bool = False) -> str:
    return compile_to(SRC, os.path.join(HERE, "liboracle.so"), verbose)


if __name__ == "__main__":
    print(build(verbose=True))
