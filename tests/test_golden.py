"""Stored fixtures under tests/golden/: a textbook worked example (Toro's
Sod star state) that pins the exact Riemann solver used by the shock-tube
pin, and a regression record of the oracle written by
tests/golden/make_golden.py (calls only oracle/)."""
import json
import os
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")


def _read_kv(path):
    out = {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = line.split()
        out[k] = float(v)
    return out


def test_exact_riemann_solver_matches_toro_sod_star_state():
    import numpy as np
    from test_oracle_scheme import _sod_exact
    ref = _read_kv(os.path.join(GOLD, "sod_star_state.txt"))
    g = 1.4
    # density just left and right of the contact at t = 0.2 (x0 = 0.5, u* t ~ 0.185)
    x = np.array([0.5 + 0.92745 * 0.2 - 1e-4, 0.5 + 0.92745 * 0.2 + 1e-4])
    rho = _sod_exact(x, 0.2, g, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    assert rho[0] == pytest.approx(ref["rho_star_left"], abs=6e-5)
    assert rho[1] == pytest.approx(ref["rho_star_right"], abs=6e-5)


def test_oracle_regression_record():
    sys.path.insert(0, GOLD)
    import make_golden
    stored = json.load(open(os.path.join(GOLD, "ot2d_128_50.json")))
    assert make_golden.record() == stored
