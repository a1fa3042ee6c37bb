"""The flop-counting build of the oracle (oracle/flopcount.py) computes the
same values as the plain build: the counting stand-in for double changes no
arithmetic.  Runs in a child process, since the oracle binding loads one
library per process."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2606_12753_amd import workloads as W  # noqa: E402

CHILD = r"""
import json, sys
sys.path.insert(0, {root!r})
from oracle import flopcount
flops = flopcount._counting_oracle()
import oracle.oracle as orc
from paper_2606_12753_amd import workloads as W
wl = W.random_smooth(n=(10, 8, 6), seed=4)
b = orc.OracleBox(wl.boxes[0])
b.set_state(wl.states[0].cons, wl.states[0].bface, 0.0)
flops.orc_flops_reset()
b.step(2)
cons, bface, t = b.get_state()
print(json.dumps({{"flops": flops.orc_flops(), "t": t,
                   "cons": [a.tobytes().hex() for a in cons],
                   "bface": [a.tobytes().hex() for a in bface]}}))
"""


def test_counting_build_matches_plain_oracle():
    out = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT)], capture_output=True,
                         text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    rec = json.loads(out.stdout.strip().splitlines()[-1])
    wl = W.random_smooth(n=(10, 8, 6), seed=4)
    b = O.OracleBox(wl.boxes[0])
    b.set_state(wl.states[0].cons, wl.states[0].bface, 0.0)
    b.step(2)
    cons, bface, t = b.get_state()
    assert rec["t"] == t
    for a, h in zip(list(cons) + list(bface), rec["cons"] + rec["bface"]):
        assert np.array_equal(a, np.frombuffer(bytes.fromhex(h), dtype=np.float64).reshape(a.shape))
    # a few thousand flops per cell-update
    assert 1000 * 480 * 2 < rec["flops"] < 10000 * 480 * 2
