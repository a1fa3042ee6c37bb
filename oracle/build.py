"""Build step of the CPU oracle (test infrastructure only).

Compiles ``mhd_oracle.c`` with gcc into ``liboracle.so`` next to this file,
and with ``mhd_oracle_cli.c`` into the command-line program ``mhd_oracle``.
FP64, no fused multiply-add contraction, IEEE division and square root;
OpenMP threads over the cell and face loops (results independent of the
thread count).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mhd_oracle.c")
CLI_SRC = os.path.join(HERE, "mhd_oracle_cli.c")
CLI = os.path.join(HERE, "mhd_oracle")
FLAGS = ["-O3", "-std=c99", "-Wall", "-Wextra", "-ffp-contract=off", "-fno-fast-math",
         "-fopenmp", "-I", HERE]
# A test may point the wrapper at a deliberately mutated build of the oracle
# (tests/test_oracle_mutations.py) through MHD_ORACLE_LIB.
LIB = os.environ.get("MHD_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")


def compile_to(src: str, lib: str, verbose: bool = False) -> str:
    cmd = ["gcc"] + FLAGS + ["-fPIC", "-shared", "-o", lib + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-D_POSIX_C_SOURCE=199309L"] + FLAGS + ["-o", CLI + ".tmp", CLI_SRC, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(CLI + ".tmp", CLI)
    return compile_to(SRC, os.path.join(HERE, "liboracle.so"), verbose)


if __name__ == "__main__":
    print(build(verbose=True))
