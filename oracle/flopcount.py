"""Floating-point operations per cell-update of the scheme, counted on the
oracle.  Test infrastructure only.

The oracle source is compiled unchanged as C++ with oracle/flopcount.hpp
force-included, which replaces double by a type that counts every +, -, *, /
and square root (one flop each; the oracle has no fused multiply-add;
negation, absolute value, min/max and comparisons count none).  One full
SSP-RK2 step of a box then gives the count per cell-update.  The values are
computed in double exactly as in the plain build.

    python oracle/flopcount.py [workload ...]
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def build(out_dir: str) -> str:
    lib = os.path.join(out_dir, "liborc_flops.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                    "-fno-fast-math", "-x", "c++", "-include",
                    os.path.join(HERE, "flopcount.hpp"), "-I", HERE, "-o", lib,
                    os.path.join(HERE, "mhd_oracle.c")], check=True)
    return lib


_FLOPS = None


def _counting_oracle():
    """The counting build, made once per process; the oracle binding loads
    the library named by MHD_ORACLE_LIB on first use, so this must run before
    anything else in the process uses the oracle."""
    global _FLOPS
    if _FLOPS is None:
        lib_path = build(tempfile.mkdtemp(prefix="orc_flops_"))
        os.environ["MHD_ORACLE_LIB"] = lib_path
        _FLOPS = C.CDLL(lib_path)
        _FLOPS.orc_flops.restype = C.c_ulonglong
    return _FLOPS


def count(workload: str = "blast_3d", n: int = 32, steps: int = 2) -> dict:
    """Flops per cell-update for `steps` steps of a workload recipe at n^3."""
    sys.path.insert(0, ROOT)
    flops = _counting_oracle()
    from paper_2606_12753_amd import workloads
    import oracle.oracle as orc
    wl = workloads.by_name(workload, n=n)
    box = orc.OracleBox(wl.boxes[0])
    box.set_state(wl.states[0].cons, wl.states[0].bface, 0.0)
    box.step(1)  # the first step's dt query and set-up are not counted
    flops.orc_flops_reset()
    box.step(steps)
    total = flops.orc_flops()
    cells = wl.boxes[0].n[0] * wl.boxes[0].n[1] * wl.boxes[0].n[2]
    counters = box.counters()
    box.close()
    return {"workload": workload, "n": n, "steps": steps,
            "flops_per_cell_update": total / (cells * steps), "counters": counters}


if __name__ == "__main__":
    for name in sys.argv[1:] or ["blast_3d", "turbulence_3d"]:
        print(count(name))
