#!/usr/bin/env python3
"""Benchmark of the ideal-MHD hot path on one MI355X.

Workload: the 3D magnetised blast wave, 256^3 periodic unit cube (seeded
+-1e-6 density noise), PLM-minmod + HLLD + CT + SSP-RK2, CFL 0.3.  A step is
one full SSP-RK2 step of the whole box (both stages, every kernel of the
path); inputs are resident in HBM before the timed region.  The timed region
is ``--steps`` graph-replayed steps on the library's stream, bracketed by HIP
events; ``value`` is cell-updates per second (cells x steps / time).

Also reported on the same line: the mixed-precision rate on the same
workload, a roofline object for the dominant kernel (algorithmic bytes per
launch over its average launch time, the latter measured with HIP events in
a separate timing pass of the same launches), and the CPU oracle's rate on a
bounded sample of the same recipe.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per cell and launch, FP64 path (compulsory reads and
# writes of each kernel's inputs and outputs, each array element once;
# stage 1 / stage 2 where they differ).  See DESIGN.md "Kernels and bytes".
BYTES_FP64 = {
    "lambda": (64, 64),
    "sweep_x": (152, 152),
    "sweep_y": (168, 168),
    "sweep_z": (168, 208),
    "ct_edge": (120, 120),
    "ct_face": (72, 96),
}
# mixed path: state FP64, work arrays FP32
BYTES_MIXED = {
    "lambda": (64, 64),
    "sweep_x": (108, 108),
    "sweep_y": (128, 128),
    "sweep_z": (156, 196),
    "ct_edge": (60, 60),
    "ct_face": (60, 84),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256, help="cells per axis of the blast box")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=128)
    ap.add_argument("--cpu-steps", type=int, default=2)
    return ap.parse_args()


def run_gpu(wl, precision, steps, warmup, flags):
    import torch
    from paper_2606_12753_amd import mhd
    spec, st = wl.boxes[0], wl.states[0]
    stream = torch.cuda.Stream()
    sim = mhd.Sim([spec], precision=precision, stream=stream.cuda_stream, flags=flags)
    sim.set_state(0, st.cons, st.bface, 0.0)
    sim.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    _, t = sim.dt(0)
    cnt = sim.counters(0)
    sim.close()
    return ms, t, cnt


def kernel_times(wl, precision, steps):
    """Average launch duration of every kernel kind, from HIP events recorded
    around each launch on the library's stream (timing pass, same launch
    configuration, no graph)."""
    import torch
    from paper_2606_12753_amd import mhd
    spec, st = wl.boxes[0], wl.states[0]
    stream = torch.cuda.Stream()
    sim = mhd.Sim([spec], precision=precision, stream=stream.cuda_stream,
                  flags=mhd.MHD_F_TIMING)
    sim.set_state(0, st.cons, st.bface, 0.0)
    sim.step(2)
    sim.kernel_times(reset=True)
    sim.step(steps)
    kt = sim.kernel_times()
    sim.close()
    return {k: (v[0] / v[1] if v[1] else 0.0, v[1]) for k, v in kt.items()}


def roofline(kt, cells, table):
    # dominant kernel = largest share of the step time
    per_step = {k: kt[k][0] * (2 if k.startswith(("sweep", "ct")) else 1) for k in table}
    dom = max(per_step, key=per_step.get)
    bytes_per_launch = 0.5 * (table[dom][0] + table[dom][1]) * cells
    avg_ms = kt[dom][0]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    return {
        "kernel": dom,
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": None,
        "avg_launch_ms": round(avg_ms, 4),
        "bytes_per_launch": int(bytes_per_launch),
    }


def cpu_baseline(n, steps):
    import oracle
    from paper_2606_12753_amd import workloads
    wl = workloads.blast_3d(n=n)
    ob = oracle.OracleBox(wl.boxes[0])
    ob.set_state(wl.states[0].cons, wl.states[0].bface)
    t0 = time.perf_counter()
    ob.step(steps)
    el = time.perf_counter() - t0
    return {
        "value": round(wl.cells * steps / el / 1e6, 4),
        "unit": "Mcell-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"blast recipe {n}^3, {steps} steps, serial FP64 oracle ({el:.1f} s)",
    }


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: this build measures one GPU only; --gpus {a.gpus} is not supported "
              "(the multi-GPU path is a design, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2606_12753_amd import mhd, workloads
    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    print(f"# building blast {a.n}^3 input", file=sys.stderr, flush=True)
    wl = workloads.blast_3d(n=a.n)
    cells = wl.cells
    flags = mhd.MHD_F_GRAPH
    print("# FP64 timed run", file=sys.stderr, flush=True)
    ms, t, cnt = run_gpu(wl, mhd.MHD_FP64, a.steps, a.warmup, flags)
    value = cells * a.steps / (ms * 1e-3) / 1e6
    print("# FP64 kernel timing pass", file=sys.stderr, flush=True)
    kt = kernel_times(wl, mhd.MHD_FP64, min(a.steps, 10))
    roof = roofline(kt, cells, BYTES_FP64)
    mixed = None
    if not a.no_mixed:
        print("# mixed timed run", file=sys.stderr, flush=True)
        ms_m, t_m, _ = run_gpu(wl, mhd.MHD_MIXED, a.steps, a.warmup, flags)
        ktm = kernel_times(wl, mhd.MHD_MIXED, min(a.steps, 10))
        mixed = {
            "value": round(cells * a.steps / (ms_m * 1e-3) / 1e6, 2),
            "ms_per_step": round(ms_m / a.steps, 4),
            "speedup_vs_fp64": round(ms / ms_m, 3),
            "roofline": roofline(ktm, cells, BYTES_MIXED),
        }
    cpu = None
    if not a.no_cpu:
        print("# CPU oracle baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(a.cpu_n, a.cpu_steps)
    line = {
        "metric": "Mcell-updates/s, FP64 vs mixed FP32 at stated L1 error; % HBM/FP64 roofline",
        "value": round(value, 2),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms / a.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"blast_3d {a.n}^3 periodic, PLM-minmod+HLLD+CT+SSP-RK2, CFL 0.3",
                   "cells": cells, "launch": "hipGraph replay per step"},
        "roofline": roof,
        "kernels_ms": {k: round(v[0], 4) for k, v in kt.items()},
        "mixed": mixed,
        "counters": cnt,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
