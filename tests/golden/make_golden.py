"""Writes tests/golden/ot2d_128_50.json: a regression record of the CPU
oracle on the 2D Orszag-Tang vortex (128^2, 50 steps).  Calls only oracle/
and the input recipes; run it again only when a change to the oracle's
arithmetic is intended, and name the passage that justifies the change."""
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2606_12753_amd import workloads  # noqa: E402


def record():
    wl = workloads.orszag_tang_2d(n=128, steps=50)
    b = oracle.OracleBox(wl.boxes[0])
    b.set_state(wl.states[0].cons, wl.states[0].bface)
    b.step(50)
    cons, bface, t = b.get_state()
    names = ["rho", "mx", "my", "mz", "E"]
    out = {"t": t.hex(), "counters": b.counters()}
    for n, a in zip(names, cons):
        out["sum_" + n] = math.fsum(a.ravel()).hex()
        out["abs_" + n] = math.fsum(abs(v) for v in a.ravel()).hex()
    for n, a in zip(["Bx", "By", "Bz"], bface):
        out["abs_" + n] = math.fsum(abs(v) for v in a.ravel()).hex()
    out["samples"] = {f"{q}:{k},{j},{i}": cons[q][k, j, i].hex()
                      for q, k, j, i in [(0, 0, 5, 7), (4, 0, 64, 64), (1, 0, 100, 3), (2, 0, 17, 90)]}
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "ot2d_128_50.json"), "w") as f:
        json.dump(record(), f, indent=1, sort_keys=True)
