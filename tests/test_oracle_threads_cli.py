"""The threaded oracle and its command-line front end: results identical for
any thread count (each cell and face is computed by one thread in the serial
order of its own terms; counters are integer sums and the time step a
maximum), and the command-line program equal to the library wrapper."""
import json
import os
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_2606_12753_amd import workloads as W

CLI = os.path.join(os.path.dirname(O.__file__), "mhd_oracle")


def run_threads(wl, steps, n, **kw):
    O.threads(n)
    b = O.OracleBox(wl.boxes[0], **kw)
    b.set_state(wl.states[0].cons, wl.states[0].bface)
    b.step(steps)
    cons, bf, t = b.get_state()
    return cons, bf, t, b.counters(), b.dt()


@pytest.mark.parametrize("wl,kw", [
    (W.random_smooth(n=(14, 11, 9), seed=71, bc=(1, 0, 1)), {}),
    (W.orszag_tang_2d(n=48), {"rk": 3, "solver": "hll", "recon": "char"}),
    (W.riemann_2d(n=40), {"limiter": "mc", "emf": "e0"}),
    (W.random_smooth(n=(10, 9, 8), seed=73, bc=(0, 1, 1)), {"emf": "uct_hll", "limiter": "vanleer"}),
])
def test_oracle_thread_count_does_not_change_results(wl, kw):
    try:
        ref = run_threads(wl, 6, 1, **kw)
        for n in (2, 5):
            got = run_threads(wl, 6, n, **kw)
            for a, b in zip(got[0] + got[1], ref[0] + ref[1]):
                assert np.array_equal(a, b), n
            assert got[2:] == ref[2:]
    finally:
        O.threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))


@pytest.mark.parametrize("flags,kw", [
    (["--rk", "3", "--recon", "char"], {"rk": 3, "recon": "char"}),
    (["--solver", "hll", "--limiter", "mc", "--emf", "uct_hll"],
     {"solver": "hll", "limiter": "mc", "emf": "uct_hll"}),
])
def test_cli_equals_wrapper(tmp_path, flags, kw):
    wl = W.random_smooth(n=(12, 10, 7), seed=72, bc=(0, 1, 0))
    spec, st = wl.boxes[0], wl.states[0]
    src, dst, rep = tmp_path / "in.bin", tmp_path / "out.bin", tmp_path / "r.json"
    O.write_state(src, spec, st.cons, st.bface, 0.0)
    n, lo, hi, bc, gamma, cfl, t, cons, bface = O.read_state(src)
    assert n == spec.n and bc == spec.bc and t == 0.0
    for a, b in zip(cons + bface, list(st.cons) + list(st.bface)):
        assert np.array_equal(a, b)
    subprocess.run([CLI, "--in", str(src), "--out", str(dst), "--steps", "5", "--threads", "3"]
                   + flags + ["--report", str(rep)], check=True)
    b = O.OracleBox(spec, **kw)
    b.set_state(st.cons, st.bface)
    b.step(5)
    oc, ob, ot = b.get_state()
    *_, t2, cons2, bface2 = O.read_state(dst)
    assert t2 == ot
    for a, c in zip(cons2 + bface2, oc + ob):
        assert np.array_equal(a, c)
    r = json.loads(rep.read_text())
    assert r["steps"] == 5 and r["t"] == ot and r["threads"] == 3
    assert r["dt_next"] == b.dt() and r["divb_max"] == b.divb_max()
    assert r["counters"] == b.counters()


def test_cli_rejects_bad_input(tmp_path):
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"NOTSTATE" + b"\0" * 64)
    p = subprocess.run([CLI, "--in", str(bad), "--out", str(tmp_path / "o"), "--steps", "1"],
                       capture_output=True, text=True)
    assert p.returncode == 2 and "not a state file" in p.stderr
    p = subprocess.run([CLI, "--steps", "1"], capture_output=True, text=True)
    assert p.returncode == 2
