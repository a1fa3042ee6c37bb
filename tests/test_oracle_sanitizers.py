"""The oracle under the host compiler's AddressSanitizer and
UndefinedBehaviorSanitizer: its command-line program, built from the same
sources with both sanitizers (aborting on the first report), runs the CPU
test inputs (periodic, outflow on each axis, 2D and 1D boxes, a blast with
pressure-floor hits and HLL fallbacks) under every scheme option without a
report, and writes the same bits as the plain build (the sanitizers change
no arithmetic: no fused multiply-add, IEEE division and square root in
both)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
from oracle import build as B
from paper_2606_12753_amd import workloads as W

pytestmark = pytest.mark.slow


@pytest.fixture(scope="module")
def sanitized_cli(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    out = str(tmp_path_factory.mktemp("asan") / "mhd_oracle_asan")
    cmd = ["gcc", "-D_POSIX_C_SOURCE=199309L", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
           "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", B.HERE, "-o", out, B.CLI_SRC, B.SRC, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer build unavailable: " + r.stderr[-500:])
    return out


def _plain_cli():
    if not os.path.exists(B.CLI) or os.path.getmtime(B.CLI) < os.path.getmtime(B.SRC):
        B.build()
    return B.CLI


CASES = [
    ("periodic", lambda: W.random_smooth(n=(11, 9, 7), seed=81), []),
    ("outflow_x", lambda: W.random_smooth(n=(9, 8, 7), seed=82, bc=(1, 0, 0)), ["--rk", "3"]),
    ("outflow_y", lambda: W.random_smooth(n=(8, 9, 7), seed=83, bc=(0, 1, 0)),
     ["--recon", "char", "--limiter", "vanleer"]),
    ("outflow_z", lambda: W.random_smooth(n=(7, 8, 9), seed=84, bc=(0, 0, 1)),
     ["--emf", "uct_hll", "--limiter", "mc"]),
    ("ot2d", lambda: W.orszag_tang_2d(n=24), ["--solver", "hll", "--emf", "e0"]),
    ("line_1d", lambda: W.cp_alfven(16, axis=1), ["--emf", "arith"]),
    ("blast_floor_hll", lambda: W.blast_3d(n=16), []),
]


@pytest.mark.parametrize("name,make,flags", CASES, ids=[c[0] for c in CASES])
def test_oracle_clean_under_sanitizers(tmp_path, sanitized_cli, name, make, flags):
    wl = make()
    spec, st = wl.boxes[0], wl.states[0]
    src = tmp_path / "in.bin"
    O.write_state(src, spec, st.cons, st.bface, 0.0)
    outs = []
    for exe in (sanitized_cli, _plain_cli()):
        dst = tmp_path / (os.path.basename(exe) + ".bin")
        env = dict(os.environ, OMP_NUM_THREADS="2",
                   ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe, "--in", str(src), "--out", str(dst), "--steps", "4"] + flags,
                           env=env, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, (name, exe, r.stderr[-3000:])
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
        outs.append(O.read_state(dst))
    (_, _, _, _, _, _, t1, c1, b1), (_, _, _, _, _, _, t2, c2, b2) = outs
    assert t1 == t2
    for a, b in zip(c1 + b1, c2 + b2):
        assert np.array_equal(a, b), name
