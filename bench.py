#!/usr/bin/env python3
"""Benchmark of the ideal-MHD hot path on one MI355X.

Workload (default): decaying MHD turbulence on the periodic unit cube at
512^3 cells (rho = 1, p = 0.6, mean B = (1, 0, 0), seeded solenoidal
Gaussian-spectrum velocity peaked at k = 4 with rms 0.5), PLM-minmod + HLLD +
CT + SSP-RK2, CFL 0.3: the largest single-GPU configuration, whose fixed step
count is 200.  ``--workload blast`` times the 256^3 magnetised blast instead.
A step is one full SSP-RK2 step of the whole box (both stages, every kernel
of the path); inputs are resident in HBM before the timed region.  The timed
region is ``--steps`` graph-replayed steps on the library's stream,
bracketed by HIP events, repeated ``--repeats`` times (each repeat re-sets
the initial state and runs ``--warmup`` untimed steps first); ``value`` is
FP64 cell-updates per second (cells x steps / median time).  The launch
variants are the autotuner's choice for the workload, fixed in
BENCH_VARIANTS so that the counter records under profiles/ describe the
kernels the line times (``--autotune`` lets the library choose again).
``fractions`` gives the step time against the per-direction design's
algorithmic bytes at 8 TB/s and against the method's compulsory traffic or
flops.

Also reported on the same line: the mixed-precision rate on the same
workload; the relative L1 error of the mixed path against the FP64 path
after the workload's fixed step count (rho, p, |B|), with max|div B| and the
drift of the mass, momentum and energy totals of both; a roofline object
for the dominant kernel (algorithmic bytes per launch over its average
launch time, measured with HIP events around each launch of a timing pass of
the same kernels on the library's stream), with its HBM traffic and VALU
issue fraction from the committed rocprofv3 records when they were taken on
the current kernel source and variant; and the CPU oracle's rate on a
bounded sample of the same recipe.

``--accuracy`` instead runs the mixed path against the FP64 path on the full
turbulence (512^3, 200 steps), ensemble (96 boxes, 100 steps) and
Kelvin-Helmholtz (768x384x384, 100 steps) workloads and prints one JSON line
per workload.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Benchmark workloads: per-axis size, fixed step count, the CPU sample's
# size and steps, and the launch variants (x, march, y segment, persistent,
# z segment) of the timed runs: the library autotuner's choice on one
# MI355X for the current kernels (bench.py --autotune prints it).
WORKLOADS = {
    "turbulence": {"n": 512, "fixed_steps": 200, "cpu_n": 160, "cpu_steps": 40,
                   "what": "turbulence_3d {n}^3 periodic, decaying solenoidal turbulence "
                           "(beta ~ 1), PLM-minmod+HLLD+CT+SSP-RK2, CFL 0.3"},
    "blast": {"n": 256, "fixed_steps": 100, "cpu_n": 256, "cpu_steps": 12,
              "what": "blast_3d {n}^3 periodic, PLM-minmod+HLLD+CT+SSP-RK2, CFL 0.3"},
    # the paper's profiled case (its Tables 2 and 5): counter records and the
    # per-kernel table; the timed line stays on the workloads above
    "orszag_tang": {"n": 352, "fixed_steps": 10, "cpu_n": 128, "cpu_steps": 4,
                    "what": "orszag_tang_3d {n}^3 periodic, PLM-minmod+HLLD+CT+SSP-RK3, CFL 0.3"},
}
BENCH_VARIANTS = {
    ("turbulence", 512): {"fp64": "0,1,64,0,64", "mixed": "0,9,128,0,128"},
    ("blast", 256): {"fp64": "0,2,64,0,64", "mixed": "2,6,16,0,128"},
    ("orszag_tang", 352): {"fp64": "1,1,32,0,16", "mixed": "1,9,32,0,128"},
}


def make_workload(name, n):
    """The benchmark input.  With BENCH_IC_CACHE set to a directory, the
    input is kept there as an .npz of its arrays (the profiler passes of one
    session then build the 512^3 input once)."""
    from paper_2606_12753_amd import workloads
    build = {"turbulence": workloads.turbulence_3d, "orszag_tang": workloads.orszag_tang_3d,
             "blast": workloads.blast_3d}[name]
    cache = os.environ.get("BENCH_IC_CACHE")
    if not cache:
        return build(n=n)
    import numpy as np
    path = os.path.join(cache, f"{name}_{n}.npz")
    if os.path.exists(path):
        z = np.load(path)
        small = build(n=8)  # the recipe's box description and metadata
        spec = type(small.boxes[0])((n, n, n), small.boxes[0].lo, small.boxes[0].hi,
                                    small.boxes[0].bc, small.boxes[0].gamma, small.boxes[0].cfl)
        st = workloads.State([z[f"c{q}"] for q in range(5)], [z[f"b{d}"] for d in range(3)], 0.0)
        return workloads.Workload(small.name, [spec], [st], small.steps, small.meta)
    wl = build(n=n)
    os.makedirs(cache, exist_ok=True)
    st = wl.states[0]
    np.savez(path, **{f"c{q}": st.cons[q] for q in range(5)},
             **{f"b{d}": st.bface[d] for d in range(3)})
    return wl


def wl_rk(wl):
    """Runge-Kutta stages of a workload (the paper's case runs three)."""
    return int(wl.meta.get("rk", 2)) if getattr(wl, "meta", None) else 2


def profile_file(kind, a, ext):
    """profiles/<kind>_<workload>_<n>.<ext>: the record of one workload."""
    return os.path.join(ROOT, "profiles", f"{kind}_{a.workload}_{a.n}.{ext}")

# Algorithmic HBM bytes per cell and launch (compulsory reads and writes of
# each kernel's inputs and outputs, each array element once; stage 1 /
# stage 2).  FP64 path:
BYTES_FP64 = {
    "sweep_x": (152, 152),    # stage 1 also reduces the CFL rate (no extra bytes)
    "sweep_y": (168, 168),
    "sweep_z": (168, 208),
    "ct_edge": (120, 120),
    "ct_face": (72, 96),
}
# mixed path: FP64 state, FP32 face fluxes, EMFs, mass fluxes and residual
BYTES_MIXED = {
    "sweep_x": (108, 108),
    "sweep_y": (116, 116),
    "sweep_z": (136, 176),
    "ct_edge": (60, 60),
    "ct_face": (60, 84),
}
# x variant 0: no x sweep; the y march reads the state once (64 B) and
# writes the cell EMF, the x- and y-face EMFs and mass fluxes and the x+y
# residual (FP64 112 B, mixed 56 B)
BYTES_FP64_FUSED = {k: v for k, v in BYTES_FP64.items() if k != "sweep_x"}
BYTES_FP64_FUSED["sweep_y"] = (176, 176)
BYTES_MIXED_FUSED = {k: v for k, v in BYTES_MIXED.items() if k != "sweep_x"}
BYTES_MIXED_FUSED["sweep_y"] = (120, 120)


def bytes_table(precision, variant):
    """Algorithmic bytes per cell of each kernel kind for a launch variant."""
    fused = variant is not None and int(variant[0]) in (0, 2)
    if precision == 0:
        return BYTES_FP64_FUSED if fused else BYTES_FP64
    return BYTES_MIXED_FUSED if fused else BYTES_MIXED


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed repeats (each re-sets the state); the median is reported")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="turbulence")
    ap.add_argument("--n", type=int, default=None,
                    help="cells per axis of the box (default: the workload's own size)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="default launch variant")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library's autotuner choose the launch variants (default: the "
                         "workload's recorded choice)")
    ap.add_argument("--fixed-steps", type=int, default=None,
                    help="steps of the accuracy runs (default: the workload's fixed count)")
    ap.add_argument("--cpu-n", type=int, default=None, help="cells per axis of the CPU sample")
    ap.add_argument("--cpu-steps", type=int, default=None, help="steps of the CPU sample")
    ap.add_argument("--cpu-threads", type=int, default=min(16, os.cpu_count() or 1),
                    help="host threads of the CPU oracle (the box's CPU share is 16)")
    ap.add_argument("--accuracy", action="store_true")
    ap.add_argument("--options", action="store_true",
                    help="the scheme options (RK3, HLL, characteristic slopes) on the benchmark input")
    ap.add_argument("--paper-workload", action="store_true",
                    help="the paper's 3D Orszag-Tang and 2D Riemann cases instead")
    ap.add_argument("--paper-case", choices=["orszag_tang_3d", "riemann_2d"], default=None,
                    help="only this one of the paper's cases")
    ap.add_argument("--ot-n", type=int, default=352, help="cells per axis of the 3D case")
    ap.add_argument("--riemann-n", type=int, default=3200, help="cells per axis of the 2D case")
    ap.add_argument("--counter-pass", action="store_true",
                    help="dispatches for a rocprofv3 --pmc run (calibration copy, then "
                         "--steps unfused steps of each precision)")
    ap.add_argument("--variant64", default=None,
                    help="x,m,segy,persistent,segz of the FP64 run (ingestion: default "
                         "from the recorded command, else 1,1,64,0,64)")
    ap.add_argument("--variant-mixed", default=None,
                    help="x,m,segy,persistent,segz of the mixed run (ingestion: default "
                         "from the recorded command, else 1,1,64,0,128)")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM traffic record from two counter-pass runs")
    ap.add_argument("--fetch-command", default="", help="command of the FETCH_SIZE run")
    ap.add_argument("--write-command", default="", help="command of the WRITE_SIZE run")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_DIR", "BENCH_LOG"),
                    help="write the kernel-trace summary from a rocprofv3 --kernel-trace "
                         "--stats run of this script")
    ap.add_argument("--trace-command", default="", help="command of the kernel-trace run")
    ap.add_argument("--ingest-sq", nargs=2, metavar=("SQ_CSV", "TRACE_DIR"),
                    help="write the SQ-counter record from a --pmc run of the counter pass and "
                         "a kernel trace of the same variants")
    ap.add_argument("--sq-command", default="", help="command of the SQ-counter run")
    ap.add_argument("--ingest-waves", metavar="SQ_CSV",
                    help="write the wave-cycle record (where the waves of each kernel spend "
                         "their cycles) from a --pmc run of the counter pass with WAVE_COUNTERS")
    ap.add_argument("--waves-command", default="", help="command of the wave-cycle run")
    ap.add_argument("--trace-out", default="kernel_trace_paper_cases.md",
                    help="file under profiles/ for the summary of a run without a bench line")
    a = ap.parse_args()
    w = WORKLOADS[a.workload]
    if a.n is None:
        a.n = w["n"]
    if a.fixed_steps is None:
        a.fixed_steps = w["fixed_steps"]
    if a.cpu_n is None:
        a.cpu_n = w["cpu_n"]
    if a.cpu_steps is None:
        a.cpu_steps = w["cpu_steps"]
    recorded = " ".join((a.fetch_command, a.write_command, a.sq_command, a.waves_command))
    fixed = BENCH_VARIANTS.get((a.workload, a.n), {})
    for attr, flag, key, default in (("variant64", "--variant64", "fp64", "1,1,64,0,64"),
                                     ("variant_mixed", "--variant-mixed", "mixed", "1,1,64,0,128")):
        if getattr(a, attr) is None:
            setattr(a, attr, variant_in_command(recorded, flag) or fixed.get(key) or default)
    return a


def variant_in_command(cmd, flag):
    """The value given to `flag` in a recorded command line, or None: counter
    records are keyed by the launch variants their runs used."""
    m = re.search(re.escape(flag) + r"\s+([0-9,]+)", cmd or "")
    return m.group(1) if m else None


SOURCES = ["csrc/mhd_kernels.hpp", "csrc/mhd_step.hpp", "csrc/mhd_lib.hip", "csrc/mhd_fp32.hip",
           "csrc/mhd_opt64.hip", "csrc/mhd_opt32.hip", "build.py"]
KINDS = ["sweep_x", "sweep_y", "sweep_z", "ct_edge", "ct_face"]
COPY_BYTES = 1 << 30  # calibration copy of the counter pass
# Floating-point operations of one cell-update (one full SSP-RK2 step of one
# cell), counted on the oracle by oracle/flopcount.py (+, -, *, /, sqrt one
# each): blast recipe 3837 at 64^3 and 3700 at 128^3, falling as 1/n with the
# share of boundary faces, so about 3630 at 256^3.
FLOPS_PER_CELL_UPDATE = 3630
FP64_PEAK_FLOPS = 78.6e12
FP32_PEAK_FLOPS = 157.3e12


def source_sha() -> str:
    """Hash of the kernel and launch sources and the build flags, comments and
    whitespace removed (counter records are only used while it matches)."""
    import re
    h = hashlib.sha256()
    for f in SOURCES:
        with open(os.path.join(ROOT, "paper_2606_12753_amd", f)) as fh:
            text = fh.read()
        if not f.endswith(".py"):
            text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
            text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def kernel_name(kind, real, variant):
    """Demangled name of the kernel a launch variant runs for a kernel kind
    on the benchmark input (x sweep: waves per SIMD; marches: waves per SIMD,
    prefetch, LDS window, LDS ring of the z march; x variants 0 and 2: the
    y march with the x faces, window in registers / LDS; then HLLD,
    primitive minmod slopes)."""
    x, m = variant[0], variant[1]
    if kind == "sweep_x":
        return f"mhd::k_sweep_x<{real}, {x}, 0, 0>"
    if kind == "sweep_y" and x in (0, 2):
        if real == "float" and x == 2:
            return f"mhd::k_sweep_march_xy<{real}, 1, 0, 256>"
        return f"mhd::k_sweep_march_xy<{real}, 0, 0, 512>"
    if kind in ("sweep_y", "sweep_z"):
        d = 1 if kind == "sweep_y" else 2
        if d == 1 and m >= 8:
            m = {8: 2, 9: 6, 10: 7}[m]
        wpe, pf, lw, cu = {1: (1, 1, 0, 0), 2: (1, 0, 0, 0), 3: (3, 0, 0, 0), 4: (4, 0, 0, 0),
                           5: (1, 1, 1, 0), 6: (1, 0, 1, 0), 7: (3, 0, 1, 0), 8: (1, 0, 0, 1),
                           9: (1, 0, 1, 1), 10: (3, 0, 1, 1)}[m]
        return f"mhd::k_sweep_march<{real}, {d}, {wpe}, {pf}, {lw}, {cu}, 0, 0, 0>"
    if kind == "ct_edge":
        # instantiated per corner average; the benchmark runs the
        # contact-upwinded one (0)
        return f"mhd::k_ct_edge<{real}, 0>"
    return f"mhd::k_{kind}<{real}>"


def launch_key(kind, real, variant):
    """What fixes a kernel's code and launch shape: its instance, the march
    segment length (marches only) and the persistent grid."""
    seg = ""
    if kind == "sweep_y":
        seg = f"|seg={variant[2]}"
    elif kind == "sweep_z":
        seg = f"|seg={variant[4] if len(variant) > 4 else variant[2]}"
    return f"{kernel_name(kind, real, variant)}{seg}|persistent={variant[3]}"


def kind_of(name):
    """(precision key, kernel kind) of a demangled kernel name, or None."""
    for real, key in (("double", "fp64"), ("float", "mixed")):
        if f"k_sweep_x<{real}," in name:
            return key, "sweep_x"
        if f"k_sweep_march<{real}, 1," in name or f"k_sweep_march_xy<{real}," in name:
            return key, "sweep_y"
        if f"k_sweep_march<{real}, 2," in name:
            return key, "sweep_z"
        if f"k_ct_edge<{real}, " in name or f"k_ct_edge<{real}>" in name:
            return key, "ct_edge"
        if f"k_ct_face<{real}>" in name:
            return key, "ct_face"
    return None


def run_gpu(wl, precision, steps, warmup, flags, repeats=1, rk=2, solver="hlld", recon="prim",
            emf="contact", limiter="minmod"):
    """Per repeat: set the initial state, `warmup` untimed steps (the first
    repeat's include the autotuner's trials), then `steps` timed steps.
    Returns the median time, every repeat's time, the final state of box 0
    and the launch variant."""
    import torch
    from paper_2606_12753_amd import mhd
    stream = torch.cuda.Stream()
    sim = mhd.Sim(wl.boxes, precision=precision, stream=stream.cuda_stream, flags=flags, rk=rk,
                  solver=solver, recon=recon, emf=emf, limiter=limiter)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(repeats):
        for b, st in enumerate(wl.states):
            sim.set_state(b, st.cons, st.bface, 0.0)
        sim.step(warmup)
        torch.cuda.synchronize()
        e0.record(stream)
        sim.step(steps)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    state = sim.get_state(0)
    ms = sorted(times)[len(times) // 2]
    out = {"ms": ms, "times": times, "state": state, "variant": sim.tuning(),
           "counters": sim.counters(0), "sim": sim}
    return out


def fractions(ms_per_step, cells, table, peak_flops, triad_gbs=None):
    """Roofline fractions of a whole step: the per-direction design's
    algorithmic bytes (every kernel, both stages) at 8 TB/s, and the method's
    compulsory state traffic (320 B per cell-update) or its flops, whichever
    bounds, over the measured step time.  With the measured triad bandwidth,
    also the design's bytes at that achievable rate (context, not a peak)."""
    t = ms_per_step * 1e-3
    nbytes = sum(b1 + b2 for b1, b2 in table.values()) * cells
    design = nbytes / (HBM_PEAK_GBS * 1e9)
    method = max(320 * cells / (HBM_PEAK_GBS * 1e9), FLOPS_PER_CELL_UPDATE * cells / peak_flops)
    out = {"design_hbm": round(design / t, 4), "method": round(method / t, 4)}
    if triad_gbs:
        out["design_vs_measured_triad"] = round(nbytes / (triad_gbs * 1e9) / t, 4)
    return out


def pcie_inclusive(wl, precision, steps, variant):
    """Cell-updates per second when the state enters from host memory and is
    read back to host memory (set_state + steps + get_state, host clock)."""
    import torch
    from paper_2606_12753_amd import mhd
    os.environ["MHD_VARIANT"] = ",".join(str(v) for v in variant)
    try:
        sim = mhd.Sim(wl.boxes, precision=precision, flags=mhd.MHD_F_GRAPH, rk=wl_rk(wl))
        st = wl.states[0]
        sim.set_state(0, st.cons, st.bface, 0.0)
        sim.step(1)
        sim.get_state(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.set_state(0, st.cons, st.bface, 0.0)
        sim.step(steps)
        sim.get_state(0)
        el = time.perf_counter() - t0
        sim.close()
    finally:
        del os.environ["MHD_VARIANT"]
    return round(wl.cells * steps / el / 1e6, 2)


def stream_bandwidth():
    """Achievable HBM bandwidth on this GPU for context: a plain device copy
    (read + write) and an a = b + s*c triad, 1 GiB operands, with torch's own
    kernels (no part of the MHD path); best of 5, GB/s of compulsory traffic."""
    import torch
    n = COPY_BYTES // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    c = torch.ones(n, dtype=torch.float64, device="cuda")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def best(fn, nbytes):
        fn()
        ms = []
        for _ in range(5):
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return round(nbytes / (min(ms) * 1e-3) / 1e9, 1)

    out = {"copy_GBs": best(lambda: a.copy_(b), 2 * COPY_BYTES),
           "triad_GBs": best(lambda: torch.add(b, c, alpha=0.5, out=a), 3 * COPY_BYTES)}
    del a, b, c
    torch.cuda.empty_cache()
    return out


def kernel_times(wl, precision, steps, variant):
    """Average launch duration of every kernel kind: HIP events recorded
    around each launch on the library's stream (timing pass with the same
    kernels and launch shapes; steps are not graph-replayed here)."""
    import torch
    from paper_2606_12753_amd import mhd
    os.environ["MHD_VARIANT"] = ",".join(str(v) for v in variant)
    try:
        stream = torch.cuda.Stream()
        sim = mhd.Sim(wl.boxes, precision=precision, stream=stream.cuda_stream,
                      flags=mhd.MHD_F_TIMING, rk=wl_rk(wl))
        for b, st in enumerate(wl.states):
            sim.set_state(b, st.cons, st.bface, 0.0)
        sim.step(2)
        sim.kernel_times(reset=True)
        sim.step(steps)
        kt = sim.kernel_times()
        sim.close()
    finally:
        del os.environ["MHD_VARIANT"]
    return {k: (v[0] / v[1] if v[1] else 0.0, v[1]) for k, v in kt.items()}


def recorded_kernel(path, precision, dom, variant):
    """The entry of a committed counter record (HBM traffic or SQ counters)
    for the dominant kernel, if the record was taken on the current kernel
    source and with the launch variant the run used; else None."""
    try:
        with open(path) as fh:
            rec = json.load(fh)
        key = "fp64" if precision == 0 else "mixed"
        real = "double" if precision == 0 else "float"
        k = rec.get(key, {}).get("kernels", {}).get(dom)
        if rec.get("source_sha") == source_sha() and k \
                and k.get("launch") == launch_key(dom, real, variant):
            return k
    except (OSError, ValueError, KeyError, TypeError):
        pass
    return None


def roofline(kt, cells, table, variant, precision, a, rk=2):
    per_step = {k: kt[k][0] * kt[k][1] for k in table}
    dom = max(per_step, key=per_step.get)
    # mean over the stages of a step: the first stage, then rk - 1 later ones
    bytes_per_launch = (table[dom][0] + (rk - 1) * table[dom][1]) / rk * cells
    avg_ms = kt[dom][0]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    k = recorded_kernel(profile_file("hbm_traffic", a, "json"), precision, dom, variant)
    traffic = int(k["bytes"]) if k else None
    sq = recorded_kernel(profile_file("sq_counters", a, "json"), precision, dom, variant)
    return {
        "kernel": dom,
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "traffic_over_algorithmic": round(traffic / bytes_per_launch, 3) if traffic else None,
        "avg_launch_ms": round(avg_ms, 4),
        "bytes_per_launch": int(bytes_per_launch),
        # share of the chip's VALU issue slots the kernel used (SQ counters;
        # FP64 and FP32 wave instructions alike) and VALU instructions per
        # wave: what bounds the FP64 sweeps before HBM does
        "valu_issue": sq["valu_issue"] if sq else None,
        "valu_per_wave": sq["valu_per_wave"] if sq else None,
    }


def derived(spec, cons, bface):
    """rho, p and |B| (cell-centred, FP64) of a state, and max|div B| both
    absolute and normalised as dx_min * max|div B| / |B|_rms."""
    import numpy as np
    bx = 0.5 * (bface[0][:, :, :-1] + bface[0][:, :, 1:])
    by = 0.5 * (bface[1][:, :-1, :] + bface[1][:, 1:, :])
    bz = 0.5 * (bface[2][:-1, :, :] + bface[2][1:, :, :])
    rho, mx, my, mz, en = cons
    b2 = bx * bx + by * by + bz * bz
    p = (spec.gamma - 1.0) * (en - 0.5 * (mx * mx + my * my + mz * mz) / rho - 0.5 * b2)
    dx = spec.dx
    div = ((bface[0][:, :, 1:] - bface[0][:, :, :-1]) / dx[0]
           + (bface[1][:, 1:, :] - bface[1][:, :-1, :]) / dx[1]
           + (bface[2][1:, :, :] - bface[2][:-1, :, :]) / dx[2])
    brms = float(np.sqrt(np.mean(b2)))
    dmax = float(np.max(np.abs(div)))
    return rho, p, np.sqrt(b2), dmax, dmax * min(dx) / max(brms, 1e-300)


def compare(spec, st64, stmx):
    import numpy as np

    def rel(a, b):
        return float(np.sum(np.abs(a - b)) / np.sum(np.abs(b)))

    r64, p64, b64, d64, n64 = derived(spec, st64[0], st64[1])
    rmx, pmx, bmx, dmx, nmx = derived(spec, stmx[0], stmx[1])
    return {"rel_l1": {"rho": rel(rmx, r64), "p": rel(pmx, p64), "|B|": rel(bmx, b64)},
            "max_divB_abs": {"fp64": d64, "mixed": dmx},
            "max_divB_norm": {"fp64": n64, "mixed": nmx}}


def cpu_baseline(a, n, steps, threads):
    """The oracle as it is (FP64, OpenMP over its cell and face loops) on a
    bounded sample of the benchmark workload: `steps` steps of the same
    recipe on n^3 cells with `threads` host threads."""
    import oracle
    wl = make_workload(a.workload, n)
    used = oracle.threads(threads)
    ob = oracle.OracleBox(wl.boxes[0])
    ob.set_state(wl.states[0].cons, wl.states[0].bface)
    t0 = time.perf_counter()
    ob.step(steps)
    el = time.perf_counter() - t0
    ob.close()
    return {
        "value": round(wl.cells * steps / el / 1e6, 4),
        "unit": "Mcell-updates/s",
        "cores": used,
        "kind": "oracle",
        "sample": f"{a.workload} recipe at {n}^3 ("
                  f"{'the benchmark input' if n == a.n else 'same seed and set-up'}), "
                  f"{steps} steps, FP64 oracle on {used} host threads, {el:.1f} s",
    }


def parse_variant(text):
    v = [int(t) for t in text.split(",")]
    if len(v) == 4:
        v.append(v[2])
    if len(v) != 5:
        raise SystemExit(f"bench.py: variant {text!r} is not x,m,seg,persistent[,segz]")
    return v


def counter_pass(a):
    """Dispatches for one rocprofv3 --pmc run: a plain device copy of 1 GiB
    (the calibration kernel: its counter reading over its known size gives
    the counter's scale), then ``--steps`` steps of each precision launched
    one by one (no graph) with the launch variants given on the command line."""
    import torch
    from paper_2606_12753_amd import mhd, workloads
    torch.cuda.set_device(0)
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    print("# counter pass: calibration copies done", file=sys.stderr, flush=True)
    wl = make_workload(a.workload, a.n)
    for prec, text in ((mhd.MHD_FP64, a.variant64), (mhd.MHD_MIXED, a.variant_mixed)):
        os.environ["MHD_VARIANT"] = ",".join(str(v) for v in parse_variant(text))
        try:
            sim = mhd.Sim(wl.boxes, precision=prec, rk=wl_rk(wl))
            for b, st in enumerate(wl.states):
                sim.set_state(b, st.cons, st.bface, 0.0)
            sim.step(a.steps)
            torch.cuda.synchronize()
            print(f"# counter pass: precision {prec} variant {sim.tuning()} done",
                  file=sys.stderr, flush=True)
            sim.close()
        finally:
            del os.environ["MHD_VARIANT"]


def read_counters(path, counter):
    """Rows (dispatch id, kernel name, value in KiB) of one counter from a
    rocprofv3 counter_collection.csv."""
    import csv
    rows = []
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    rows.sort()
    return rows


def ingest_counters(a):
    """Writes the HBM traffic record from the FETCH_SIZE and WRITE_SIZE runs
    of the counter pass: the three largest runtime copy dispatches are the
    1 GiB calibration copies; each counter is scaled by the copy's known size
    over its reading; per kernel kind, KiB per dispatch averaged over the
    dispatches of the run (both RK stages)."""
    fetch_csv, write_csv = a.ingest_counters
    out = {"workload": f"{a.workload} {a.n}^3", "source_sha": source_sha(),
           "commands": {"fetch": a.fetch_command, "write": a.write_command},
           "calibration": {"copy_bytes": COPY_BYTES}}
    per = {}
    scale = {}
    for name, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"),
                                ("write", write_csv, "WRITE_SIZE")):
        rows = read_counters(path, counter)
        copies = sorted(v for _, k, v in rows if k == "__amd_rocclr_copyBuffer")[-3:]
        if len(copies) < 3:
            raise SystemExit(f"bench.py: {path}: calibration copies not found")
        mean = sum(copies) / 3
        scale[name] = round(COPY_BYTES / 1024 / mean, 3)
        out["calibration"][f"{counter}_kib"] = round(mean, 1)
        for _, k, v in rows:
            kk = kind_of(k)
            if kk is None:
                continue
            rec = per.setdefault(kk, {"names": set(), "fetch": [], "write": []})
            rec["names"].add(k)
            rec[name].append(v)
    out["scale"] = scale
    for key, text in (("fp64", a.variant64), ("mixed", a.variant_mixed)):
        algo = bytes_table(0 if key == "fp64" else 1, parse_variant(text))
        cells = a.n ** 3
        kernels = {}
        for kind in KINDS:
            rec = per.get((key, kind))
            if not rec or not rec["fetch"] or not rec["write"]:
                continue
            f = sum(rec["fetch"]) / len(rec["fetch"])
            w = sum(rec["write"]) / len(rec["write"])
            byts = (f * scale["fetch"] + w * scale["write"]) * 1024
            rk = 3 if a.workload == "orszag_tang" else 2
            alg = (algo[kind][0] + (rk - 1) * algo[kind][1]) / rk * cells
            real = "double" if key == "fp64" else "float"
            kernels[kind] = {"launch": launch_key(kind, real, parse_variant(text)),
                             "kernel": sorted(rec["names"]), "dispatches": len(rec["fetch"]),
                             "fetch_kib": round(f, 1), "write_kib": round(w, 1),
                             "bytes": int(byts), "algorithmic_bytes": int(alg),
                             "ratio": round(byts / alg, 3)}
        out[key] = {"variant": parse_variant(text), "kernels": kernels}
    with open(profile_file("hbm_traffic", a, "json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps({k: {kk: v["ratio"] for kk, v in out[k]["kernels"].items()}
                      for k in ("fp64", "mixed")}))


VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4   # wave64 VALU instructions per second (4 cycles each)
SQ_COUNTERS = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
               "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_BUSY_CYCLES"]


def ingest_sq(a):
    """Writes the instruction-level record of the benchmark's kernels from
    one rocprofv3 --pmc run of the counter pass (the SQ_COUNTERS) and a
    kernel trace of the same launch variants: per kernel, VALU instructions
    per wave, VALU issue rate against the chip's issue ceiling (256 CUs x 4
    SIMDs x 2.4 GHz, 4 cycles per wave64 instruction), LDS bank-conflict
    cycles per LDS instruction, and the registers, LDS and scratch of its
    code object."""
    import csv
    sq_csv, tdir = a.ingest_sq
    per = {}
    with open(sq_csv, newline="") as fh:
        for r in csv.DictReader(fh):
            k = kind_of(r["Kernel_Name"])
            if k is None:
                continue
            rec = per.setdefault((k, r["Kernel_Name"]), {})
            rec.setdefault(r["Counter_Name"], {}).setdefault(int(r["Dispatch_Id"]), 0.0)
            rec[r["Counter_Name"]][int(r["Dispatch_Id"])] += float(r["Counter_Value"])
    dur, res = {}, {}
    with open(os.path.join(tdir, "run_kernel_trace.csv"), newline="") as fh:
        for r in csv.DictReader(fh):
            n = r["Kernel_Name"]
            dur.setdefault(n, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
            res[n] = (r.get("VGPR_Count") or r.get("Arch_VGPR_Count"), r["SGPR_Count"],
                      r["LDS_Block_Size"], r["Scratch_Size"])
    lines = [f"# SQ counters: {a.workload} {a.n}^3, the benchmark's kernels", "",
             "Commands (from the repository root):", "", "```", a.sq_command, a.trace_command, "```",
             "", f"Kernel source hash {source_sha()}; variants FP64 {a.variant64}, mixed "
             f"{a.variant_mixed}.  VALU issue = SQ_INSTS_VALU / (duration x "
             f"{VALU_ISSUE_PER_S / 1e9:.0f} G wave-instructions/s), the fraction of the chip's "
             "VALU issue slots used; durations are the trace's averages for the kernel in this "
             "unfused counter pass (longer than the graph-replayed bench's).  VGPR_Count, "
             "SGPR_Count, LDS and scratch are rocprofv3's per-dispatch fields (VGPR_Count is half "
             "the compiler's register count on this target: 72 for the FP64 x sweep's 142).", "",
             "| precision | kernel | waves | VALU / wave | SALU / wave | VMEM rd / wave | "
             "LDS / wave | LDS conflict cycles / LDS instr | avg us | algorithmic GB/s | "
             "VALU issue | VGPR_Count | SGPR_Count | LDS bytes | scratch bytes |",
             "|---|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    rk = 3 if a.workload == "orszag_tang" else 2
    cells = a.n ** 3
    record = {"workload": f"{a.workload} {a.n}^3", "source_sha": source_sha(),
              "commands": {"sq": a.sq_command, "trace": a.trace_command}}
    for key, text in (("fp64", a.variant64), ("mixed", a.variant_mixed)):
        record[key] = {"variant": parse_variant(text), "kernels": {}}
    for ((key, kind), name), rec in sorted(per.items(), key=lambda x: (x[0][0][0], KINDS.index(x[0][0][1]))):
        def mean(c):
            v = rec.get(c, {})
            return sum(v.values()) / len(v) if v else float("nan")
        waves = mean("SQ_WAVES")
        valu = mean("SQ_INSTS_VALU")
        lds = mean("SQ_INSTS_LDS")
        d = dur.get(name)
        avg = sum(d) / len(d) if d else float("nan")
        issue = valu / (avg * VALU_ISSUE_PER_S) if d else float("nan")
        vg, sg, lb, sc = res.get(name, ("-", "-", "-", "-"))
        conf = mean("SQ_LDS_BANK_CONFLICT") / lds if lds > 0 else 0.0
        algo = bytes_table(0 if key == "fp64" else 1, record[key]["variant"])[kind]
        gbs = (algo[0] + (rk - 1) * algo[1]) / rk * cells / avg / 1e9 if d else float("nan")
        lines.append(f"| {key} | `{name.replace('void ', '').replace('(mhd::Launch)', '')}` | "
                     f"{waves:.0f} | {valu / waves:.0f} | {mean('SQ_INSTS_SALU') / waves:.0f} | "
                     f"{mean('SQ_INSTS_VMEM_RD') / waves:.1f} | {lds / waves:.1f} | {conf:.3f} | "
                     f"{avg * 1e6:.1f} | {gbs:.0f} | {issue:.2f} | {vg} | {sg} | {lb} | {sc} |")
        real = "double" if key == "fp64" else "float"
        variant = record[key]["variant"]
        if kernel_name(kind, real, variant) in name:
            record[key]["kernels"][kind] = {
                "launch": launch_key(kind, real, variant), "kernel": name,
                "valu_per_wave": round(valu / waves, 1), "valu_issue": round(issue, 3),
                "lds_conflict_per_instr": round(conf, 4), "avg_us_unfused": round(avg * 1e6, 1),
                "vgpr_count": vg, "scratch_bytes": sc}
    if a.workload == "orszag_tang":
        lines += ["", "Context, not a target: the paper's own kernel table for this case on one "
                  "MI250X GCD (its Table 5, section 3.2; OpenMP, FP64, one direction of one "
                  "stage per invocation, unified memory), time / memory bandwidth / VGPRs per "
                  "wavefront / scratch / VALU utilisation: HLLD_i 29.7 ms / 566 GB/s / 120 / 32 B "
                  "/ 15%; HLLD_j,k 110.6 ms / 248 GB/s / 108 / 32 B / 4%; Reconstruct 25.7 ms / "
                  "417 GB/s / 92 / 32 B / 58%; RightHandSide 35.0 ms / 447 GB/s / 88 / 32 B / 3%; "
                  "CT_EMF 32.4 ms / 717 GB/s / 88 / 32 B / 0.3%; US 119.8 ms / 290 GB/s / 56 / "
                  "32 B / 4%.  Here reconstruction, Riemann solve and flux divergence of a "
                  "direction are one kernel (the x sweep, the y and z marches), CT_EMF is the "
                  "corner-EMF kernel and the face update with the stage combine is the "
                  "face kernel; the algorithmic GB/s count each kernel's compulsory bytes once."]
    with open(profile_file("sq_counters", a, "md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(profile_file("sq_counters", a, "json"), "w") as fh:
        json.dump(record, fh, indent=1)
        fh.write("\n")
    print("\n".join(lines))


# one --pmc pass: cycles of the resident waves and what they were doing
WAVE_COUNTERS = ("SQ_WAVE_CYCLES", "SQ_ACTIVE_INST_VALU", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY",
                 "SQ_ACTIVE_INST_LDS", "SQ_WAIT_INST_LDS")


def ingest_waves(a):
    """Writes where the waves of each of the benchmark's kernels spend their
    cycles, from one rocprofv3 --pmc run of the counter pass with
    WAVE_COUNTERS: each counter summed over the kernel's dispatches, as a
    fraction of the summed wave-cycles.  A wave can be issuing one
    instruction while waiting on another, so the fractions need not add
    up to one."""
    import csv
    per = {}
    with open(a.ingest_waves, newline="") as fh:
        for r in csv.DictReader(fh):
            k = kind_of(r["Kernel_Name"])
            if k is None or r["Counter_Name"] not in WAVE_COUNTERS:
                continue
            rec = per.setdefault((k, r["Kernel_Name"]), {})
            rec[r["Counter_Name"]] = rec.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    lines = [f"# Wave cycles: {a.workload} {a.n}^3, the benchmark's kernels", "",
             "Command (from the repository root):", "", "```", a.waves_command, "```", "",
             f"Kernel source hash {source_sha()}; variants FP64 {a.variant64}, mixed "
             f"{a.variant_mixed}.  Each column is a counter summed over the kernel's dispatches "
             "divided by SQ_WAVE_CYCLES summed the same way: SQ_ACTIVE_INST_VALU (a VALU "
             "instruction in flight), SQ_WAIT_ANY (waiting on a memory counter or a barrier), "
             "SQ_WAIT_INST_ANY (waiting to issue: dependencies and arbitration), "
             "SQ_ACTIVE_INST_LDS and SQ_WAIT_INST_LDS.  A wave can issue while it waits on "
             "an earlier load, so the columns need not add up to one.", "",
             "| precision | kernel | VALU active | waiting (memory, barrier) | waiting to issue | "
             "LDS active | LDS issue wait |",
             "|---|---|---:|---:|---:|---:|---:|"]
    record = {"workload": f"{a.workload} {a.n}^3", "source_sha": source_sha(),
              "command": a.waves_command, "fp64": {}, "mixed": {}}
    for ((key, kind), name), rec in sorted(per.items(), key=lambda x: (x[0][0][0], KINDS.index(x[0][0][1]))):
        cyc = rec.get("SQ_WAVE_CYCLES", 0.0)
        if cyc <= 0:
            continue
        f = {c: rec.get(c, 0.0) / cyc for c in WAVE_COUNTERS[1:]}
        lines.append(f"| {key} | `{name.replace('void ', '').replace('(mhd::Launch)', '')}` | "
                     + " | ".join(f"{f[c]:.2f}" for c in WAVE_COUNTERS[1:]) + " |")
        record[key][name] = {c: round(v, 4) for c, v in f.items()}
    with open(profile_file("sq_wave_cycles", a, "md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(profile_file("sq_wave_cycles", a, "json"), "w") as fh:
        json.dump(record, fh, indent=1)
        fh.write("\n")
    print("\n".join(lines))


def summarize_trace(a):
    """Writes the kernel-trace summary: rocprofv3's per-kernel statistics and,
    for the dominant kernel of each precision, the average duration of the
    dispatches with the launch shape the bench chose, beside the bench's own
    HIP-event average."""
    import csv
    tdir, log = a.summarize_trace
    bench = None
    cases = []
    with open(log) as fh:
        for line in fh:
            if line.startswith('{"metric"'):
                bench = json.loads(line)
            elif line.startswith('{"workload"'):
                cases.append(json.loads(line))
    if bench is None:
        if not cases:
            raise SystemExit(f"bench.py: no bench or workload line in {log}")
        return summarize_case_trace(a, tdir, cases)
    stats = []
    with open(os.path.join(tdir, "run_kernel_stats.csv"), newline="") as fh:
        for r in csv.DictReader(fh):
            stats.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                          float(r["Percentage"])))
    trace = {}
    with open(os.path.join(tdir, "run_kernel_trace.csv"), newline="") as fh:
        for r in csv.DictReader(fh):
            key = (r["Kernel_Name"], int(r["Grid_Size_X"]))
            trace.setdefault(key, []).append(
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines = [f"# rocprofv3 kernel trace: {a.workload} {a.n}^3, FP64 and mixed", "",
             "Command (from the repository root):", "", "```", a.trace_command, "```", "",
             f"Kernel source hash {bench.get('source_sha')}; bench line: FP64 "
             f"{bench['value']} Mcell-updates/s, variant {bench['config']['variant']}"
             + (f"; mixed {bench['mixed']['value']} Mcell-updates/s, variant "
                f"{bench['mixed']['variant']}" if bench.get("mixed") else "") + ".", "",
             "| kernel | calls | avg us | % time |", "|---|---:|---:|---:|"]
    for name, calls, avg, pct in stats[:16]:
        lines.append(f"| `{name}` | {calls} | {avg:.1f} | {pct:.2f} |")
    lines += ["", "Dominant kernel, launches of the bench's launch shape (rocprofv3) against "
              "the bench's HIP-event average:", "",
              "| precision | kernel | grid threads | dispatches | rocprofv3 avg us | "
              "bench avg us | ratio |", "|---|---|---:|---:|---:|---:|---:|"]
    for key, real, blk in (("fp64", "double", bench), ("mixed", "float", bench.get("mixed"))):
        if not blk:
            continue
        roof = blk["roofline"]
        variant = blk["config"]["variant"] if key == "fp64" else blk["variant"]
        want = kernel_name(roof["kernel"], real, variant)
        groups = [(len(v), g, v) for (n, g), v in trace.items() if want in n]
        if not groups:
            lines.append(f"| {key} | `{want}` | - | 0 | - | {roof['avg_launch_ms'] * 1e3:.1f} | - |")
            continue
        cnt, grid, durs = max(groups)
        avg = sum(durs) / cnt
        bench_us = roof["avg_launch_ms"] * 1e3
        lines.append(f"| {key} | `{want}` | {grid} | {cnt} | {avg:.1f} | {bench_us:.1f} | "
                     f"{avg / bench_us:.3f} |")
    with open(profile_file("kernel_trace", a, "md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_case_trace(a, tdir, cases):
    """Kernel-trace summary of a --paper-workload (or --options) run: the
    per-kernel statistics of rocprofv3 and the timed results of the run."""
    import csv
    stats = []
    with open(os.path.join(tdir, "run_kernel_stats.csv"), newline="") as fh:
        for r in csv.DictReader(fh):
            stats.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                          float(r["Percentage"])))
    lines = [f"# rocprofv3 kernel trace: {', '.join(c['workload'].split(',')[0] for c in cases)}",
             "", "Command (from the repository root):", "", "```", a.trace_command, "```", "",
             f"Kernel source hash {source_sha()}.", "",
             "| workload | FP64 s / 10 steps (Mcell-updates/s) | mixed s / 10 steps (Mcell-updates/s) |",
             "|---|---:|---:|"]
    for c in cases:
        if "fp64" in c and "s_10_steps" in c["fp64"]:
            lines.append(f"| {c['workload']} | {c['fp64']['s_10_steps']} "
                         f"({c['fp64']['Mcell_updates_per_s']}) | {c['mixed']['s_10_steps']} "
                         f"({c['mixed']['Mcell_updates_per_s']}) |")
    lines += ["", "| kernel | calls | avg us | % time |", "|---|---:|---:|---:|"]
    for name, calls, avg, pct in stats[:24]:
        lines.append(f"| `{name}` | {calls} | {avg:.1f} | {pct:.2f} |")
    out = os.path.join(ROOT, "profiles", a.trace_out)
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


# The paper's Figure 1: wall time of 10 steps of its 3D Orszag-Tang run on
# 352^3 cells (whole application, third-order Runge-Kutta), by hardware and
# programming model; Table 3: one invocation (one direction, one stage) of
# its reconstruction and HLL kernels on the 3200^2 2D Riemann problem, A100.
# Context only: other hardware, other code.
PAPER_OT3D_10_STEPS_S = {"A100, OpenACC": 13.9, "A100, OpenMP": 17.2,
                         "MI250X (one GCD), OpenMP": 48.1}
PAPER_RIEMANN2D_INVOCATION_MS = {"Reconstruct, A100 OpenACC": 1.24,
                                 "Reconstruct, A100 OpenMP": 58.0,
                                 "HLL, A100 OpenACC": 1.63, "HLL, A100 OpenMP": 9.84}


def kernel_times_of(wl, precision, steps, variant, rk, solver, recon="prim", emf="contact",
                    limiter="minmod"):
    """kernel_times for a given integrator, Riemann solver and reconstruction."""
    import torch
    from paper_2606_12753_amd import mhd
    os.environ["MHD_VARIANT"] = ",".join(str(v) for v in variant)
    try:
        stream = torch.cuda.Stream()
        sim = mhd.Sim(wl.boxes, precision=precision, stream=stream.cuda_stream,
                      flags=mhd.MHD_F_TIMING, rk=rk, solver=solver, recon=recon, emf=emf,
                      limiter=limiter)
        for b, st in enumerate(wl.states):
            sim.set_state(b, st.cons, st.bface, 0.0)
        sim.step(1)
        sim.kernel_times(reset=True)
        sim.step(steps)
        kt = sim.kernel_times()
        sim.close()
    finally:
        del os.environ["MHD_VARIANT"]
    return {k: round(v[0] / v[1], 4) for k, v in kt.items() if v[1]}


def paper_workload(a, flags):
    """The paper's two profiled cases on this library, FP64 and mixed, 10
    steps each, median of three timed repeats: the 3D Orszag-Tang vortex on
    352^3 cells (HLLD, SSP-RK3) and the thin 2D Riemann problem on 3200^2
    cells (HLL, SSP-RK3), with per-launch kernel times (ms) of each."""
    from paper_2606_12753_amd import mhd, workloads
    cases = [("orszag_tang_3d", lambda: workloads.orszag_tang_3d(n=a.ot_n, steps=10), "hlld",
              f"orszag_tang_3d {a.ot_n}^3, SSP-RK3, 10 steps, PLM-minmod+HLLD+CT, CFL 0.3",
              {"paper_s_10_steps": PAPER_OT3D_10_STEPS_S}),
             ("riemann_2d", lambda: workloads.riemann_2d(n=a.riemann_n, steps=10), "hll",
              f"riemann_2d {a.riemann_n}x{a.riemann_n}x1, SSP-RK3, 10 steps, PLM-minmod+HLL+CT, CFL 0.4",
              {"paper_ms_per_invocation": PAPER_RIEMANN2D_INVOCATION_MS})]
    for name, make, solver, desc, ctx in cases:
        if a.paper_case and name != a.paper_case:
            continue
        print(f"# paper workload: building {name}", file=sys.stderr, flush=True)
        wl = make()
        res = {}
        for prec, key in ((mhd.MHD_FP64, "fp64"), (mhd.MHD_MIXED, "mixed")):
            print(f"# paper workload: {name} {key}", file=sys.stderr, flush=True)
            r = run_gpu(wl, prec, 10, 2, flags, repeats=3, rk=3, solver=solver)
            r["sim"].close()
            r["kernels_ms"] = kernel_times_of(wl, prec, 3, r["variant"], 3, solver)
            res[key] = r
        out = {"workload": desc, "cells": wl.cells}
        for key in ("fp64", "mixed"):
            r = res[key]
            out[key] = {"s_10_steps": round(r["ms"] * 1e-3, 4),
                        "Mcell_updates_per_s": round(wl.cells * 10 / (r["ms"] * 1e-3) / 1e6, 1),
                        "variant": r["variant"], "kernels_ms_per_launch": r["kernels_ms"]}
        out["speedup_mixed"] = round(res["fp64"]["ms"] / res["mixed"]["ms"], 3)
        out.update(ctx)
        out.update(compare(wl.boxes[0], res["fp64"]["state"], res["mixed"]["state"]))
        print(json.dumps(out), flush=True)
        del wl, res


def options_bench(a, flags):
    """Cost of the scheme options on the benchmark input (blast, n^3): the
    default (primitive slopes, HLLD, SSP-RK2, contact-upwinded corner EMFs)
    against SSP-RK3, HLL at every face, characteristic slopes, the E0,
    arithmetic and upwind-CT corner EMFs and the MC and van Leer limiters,
    FP64 and mixed; median of three repeats of a.steps steps, per-launch
    kernel times, and the x sweep's algorithmic HBM rate (its bytes do not
    depend on the options; the upwind CT adds the stores of the face wave
    speeds)."""
    from paper_2606_12753_amd import mhd, workloads
    print(f"# options: building {a.workload} {a.n}^3 input", file=sys.stderr, flush=True)
    wl = make_workload(a.workload, a.n)
    cells = wl.cells
    opts = [("default", dict(rk=2, solver="hlld", recon="prim", emf="contact")),
            ("rk3", dict(rk=3, solver="hlld", recon="prim", emf="contact")),
            ("hll", dict(rk=2, solver="hll", recon="prim", emf="contact")),
            ("char", dict(rk=2, solver="hlld", recon="char", emf="contact")),
            ("emf_e0", dict(rk=2, solver="hlld", recon="prim", emf="e0")),
            ("emf_arith", dict(rk=2, solver="hlld", recon="prim", emf="arith")),
            ("emf_uct_hll", dict(rk=2, solver="hlld", recon="prim", emf="uct_hll")),
            ("limiter_mc", dict(rk=2, solver="hlld", recon="prim", emf="contact", limiter="mc")),
            ("limiter_vanleer", dict(rk=2, solver="hlld", recon="prim", emf="contact",
                                     limiter="vanleer"))]
    out = {"workload": f"{a.workload} {a.n}^3 periodic, PLM-minmod+CT, CFL 0.3", "cells": cells,
           "steps": a.steps, "options": {}}
    for name, kw in opts:
        row = {}
        for prec, key in ((mhd.MHD_FP64, "fp64"), (mhd.MHD_MIXED, "mixed")):
            print(f"# options: {name} {key}", file=sys.stderr, flush=True)
            r = run_gpu(wl, prec, a.steps, a.warmup, flags, repeats=3, **kw)
            r["sim"].close()
            kt = kernel_times_of(wl, prec, min(a.steps, 10), r["variant"], kw["rk"], kw["solver"],
                                 kw["recon"], kw["emf"], kw.get("limiter", "minmod"))
            table = bytes_table(prec, r["variant"])
            xk = "sweep_x" if "sweep_x" in table and kt.get("sweep_x") else "sweep_y"
            xbytes = 0.5 * (table[xk][0] + table[xk][1]) * cells
            row[key] = {"Mcell_updates_per_s": round(cells * a.steps / (r["ms"] * 1e-3) / 1e6, 1),
                        "ms_per_step": round(r["ms"] / a.steps, 4), "variant": r["variant"],
                        "kernels_ms_per_launch": kt,
                        f"{xk}_hbm_frac": round(xbytes / (kt[xk] * 1e-3) / 1e9
                                                / HBM_PEAK_GBS, 4)}
        row["speedup_mixed"] = round(row["mixed"]["Mcell_updates_per_s"]
                                     / row["fp64"]["Mcell_updates_per_s"], 3)
        out["options"][name] = row
    print(json.dumps(out), flush=True)


def accuracy(flags):
    """Mixed against FP64 on the full-size secondary workloads."""
    from paper_2606_12753_amd import mhd, workloads
    for name, kw in (("turbulence_3d", {}), ("ensemble", {}), ("kelvin_helmholtz", {})):
        print(f"# accuracy: building {name}", file=sys.stderr, flush=True)
        wl = workloads.by_name(name, **kw)
        steps = wl.steps
        res = {}
        for prec in (mhd.MHD_FP64, mhd.MHD_MIXED):
            print(f"# accuracy: {name} precision {prec}", file=sys.stderr, flush=True)
            r = run_gpu(wl, prec, steps - 1, 1, flags)
            sim = r["sim"]
            states = [sim.get_state(b) for b in range(len(wl.boxes))]
            sim.close()
            res[prec] = (r["ms"], states, r["variant"])
        out = {"workload": name, "cells": wl.cells, "steps": steps, "boxes": len(wl.boxes)}
        for prec, key in ((mhd.MHD_FP64, "fp64"), (mhd.MHD_MIXED, "mixed")):
            ms = res[prec][0]
            out[key] = {"Mcell_updates_per_s": round(wl.cells * (steps - 1) / (ms * 1e-3) / 1e6, 1),
                        "variant": res[prec][2]}
        out["speedup"] = round(res[mhd.MHD_FP64][0] / res[mhd.MHD_MIXED][0], 3)
        # error of the mixed run per box, worst box reported
        worst = None
        for b, spec in enumerate(wl.boxes):
            c = compare(spec, res[mhd.MHD_FP64][1][b], res[mhd.MHD_MIXED][1][b])
            if worst is None or max(c["rel_l1"].values()) > max(worst["rel_l1"].values()):
                worst = c
        out.update(worst)
        # totals of mass, momentum and energy, worst box per quantity: drift
        # from the initial state (conservation where every axis is periodic;
        # with outflow walls it includes what left through them), and the
        # mixed run's totals against the FP64 run's
        periodic = all(all(bc == workloads.PERIODIC for bc in spec.bc) for spec in wl.boxes)
        dr = {"fp64": {}, "mixed": {}}
        tot = {}
        for b in range(len(wl.boxes)):
            for prec, key in ((mhd.MHD_FP64, "fp64"), (mhd.MHD_MIXED, "mixed")):
                for q, v in drift(wl.states[b].cons, res[prec][1][b][0]).items():
                    dr[key][q] = max(dr[key].get(q, 0.0), v)
            for q, v in drift(res[mhd.MHD_FP64][1][b][0], res[mhd.MHD_MIXED][1][b][0]).items():
                tot[q] = max(tot.get(q, 0.0), v)
        out["totals_drift_from_initial"] = dict(dr, periodic=periodic)
        out["mixed_totals_vs_fp64"] = tot
        print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.ingest_counters:
        ingest_counters(a)
        return
    if a.summarize_trace:
        summarize_trace(a)
        return
    if a.ingest_sq:
        ingest_sq(a)
        return
    if a.ingest_waves:
        ingest_waves(a)
        return
    if a.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {a.gpus} is not supported "
              "(sharding across GPUs is designed, not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2606_12753_amd import mhd, workloads
    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if a.counter_pass:
        counter_pass(a)
        return
    flags = mhd.MHD_F_GRAPH | (0 if a.no_tune else mhd.MHD_F_AUTOTUNE)
    if a.accuracy:
        accuracy(flags)
        return
    if a.paper_workload:
        paper_workload(a, flags)
        return
    if a.options:
        options_bench(a, flags)
        return
    print(f"# building {a.workload} {a.n}^3 input", file=sys.stderr, flush=True)
    wl = make_workload(a.workload, a.n)
    spec = wl.boxes[0]
    cells = wl.cells
    print("# HBM stream reference", file=sys.stderr, flush=True)
    stream = stream_bandwidth()
    fixed = {}
    if not a.autotune and not a.no_tune:
        fixed = {mhd.MHD_FP64: parse_variant(a.variant64), mhd.MHD_MIXED: parse_variant(a.variant_mixed)}
        flags = mhd.MHD_F_GRAPH
    print("# FP64 timed run", file=sys.stderr, flush=True)
    rk = wl_rk(wl)
    r64 = with_variant(fixed.get(mhd.MHD_FP64), run_gpu, wl, mhd.MHD_FP64, a.steps, a.warmup,
                       flags, a.repeats, rk=rk)
    r64["sim"].close()
    ms = r64["ms"]
    value = cells * a.steps / (ms * 1e-3) / 1e6
    print("# FP64 kernel timing pass", file=sys.stderr, flush=True)
    kt = kernel_times(wl, mhd.MHD_FP64, min(a.steps, 10), r64["variant"])
    t64 = bytes_table(mhd.MHD_FP64, r64["variant"])
    roof = roofline(kt, cells, t64, r64["variant"], mhd.MHD_FP64, a, rk)
    print("# FP64 PCIe-inclusive run", file=sys.stderr, flush=True)
    pcie = pcie_inclusive(wl, mhd.MHD_FP64, a.steps, r64["variant"])
    mixed = None
    print(f"# FP64 run over the fixed step count ({a.fixed_steps})", file=sys.stderr, flush=True)
    s64, cnt64 = fixed_run(wl, mhd.MHD_FP64, a.fixed_steps, r64["variant"])
    drift64 = drift(wl.states[0].cons, s64[0])
    if not a.no_mixed:
        print("# mixed timed run", file=sys.stderr, flush=True)
        rmx = with_variant(fixed.get(mhd.MHD_MIXED), run_gpu, wl, mhd.MHD_MIXED, a.steps,
                           a.warmup, flags, a.repeats, rk=rk)
        rmx["sim"].close()
        ktm = kernel_times(wl, mhd.MHD_MIXED, min(a.steps, 10), rmx["variant"])
        print(f"# mixed run over the fixed step count ({a.fixed_steps})", file=sys.stderr,
              flush=True)
        smx, cntmx = fixed_run(wl, mhd.MHD_MIXED, a.fixed_steps, rmx["variant"])
        acc = compare(spec, s64, smx)
        mixed = {
            "value": round(cells * a.steps / (rmx["ms"] * 1e-3) / 1e6, 2),
            "ms_per_step": round(rmx["ms"] / a.steps, 4),
            "speedup_vs_fp64": round(ms / rmx["ms"], 3),
            "ms_per_step_repeats": [round(t / a.steps, 4) for t in rmx["times"]],
            "fractions": fractions(rmx["ms"] / a.steps, cells,
                                   bytes_table(mhd.MHD_MIXED, rmx["variant"]), FP32_PEAK_FLOPS,
                                   stream["triad_GBs"]),
            "accuracy_vs_fp64": acc,
            "after_steps": a.fixed_steps,
            "conservation_drift": drift(wl.states[0].cons, smx[0]),
            "counters": cntmx,
            "variant": rmx["variant"],
            "roofline": roofline(ktm, cells, bytes_table(mhd.MHD_MIXED, rmx["variant"]),
                                 rmx["variant"], mhd.MHD_MIXED, a, rk),
            "kernels_ms": {k: round(v[0], 4) for k, v in ktm.items() if v[1]},
        }
        del smx
    del s64
    cpu = None
    if not a.no_cpu:
        print("# CPU oracle baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(a, a.cpu_n, a.cpu_steps, a.cpu_threads)
    line = {
        "metric": "Mcell-updates/s, FP64 vs mixed FP32 at stated L1 error; % HBM/FP64 roofline",
        "value": round(value, 2),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms / a.steps, 4),
        "repeats": a.repeats,
        "ms_per_step_repeats": [round(t / a.steps, 4) for t in r64["times"]],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[a.workload]["what"].format(n=a.n),
                   "cells": cells, "launch": "hipGraph replay per step",
                   "variant": r64["variant"],
                   "variant_source": "autotuned in this run" if not fixed
                   else "the workload's recorded autotuner choice",
                   "fixed_steps": a.fixed_steps},
        "roofline": roof,
        "fractions": fractions(ms / a.steps, cells, t64, FP64_PEAK_FLOPS,
                               stream["triad_GBs"]),
        "kernels_ms": {k: round(v[0], 4) for k, v in kt.items() if v[1]},
        "conservation_drift": drift64,
        "counters": cnt64,
        "mixed": mixed,
        "hbm_stream": stream,
        "pcie_inclusive": {"value": pcie, "unit": "Mcell-updates/s",
                           "what": f"host set_state + {a.steps} steps + host get_state, FP64"},
        "cpu_baseline": cpu,
        "source_sha": source_sha(),
    }
    print(json.dumps(line), flush=True)


def with_variant(variant, fn, *args, **kw):
    """fn(*args) with the library's launch variant fixed (MHD_VARIANT) when
    variant is given, else as the flags choose."""
    if variant is None:
        return fn(*args, **kw)
    os.environ["MHD_VARIANT"] = ",".join(str(v) for v in variant)
    try:
        return fn(*args, **kw)
    finally:
        del os.environ["MHD_VARIANT"]


def fixed_run(wl, precision, steps, variant):
    """The workload's state after its fixed step count (graph replay, the
    timed run's variant) and the event counters of box 0."""
    from paper_2606_12753_amd import mhd

    def go():
        with mhd.Sim(wl.boxes, precision=precision, flags=mhd.MHD_F_GRAPH, rk=wl_rk(wl)) as sim:
            for b, st in enumerate(wl.states):
                sim.set_state(b, st.cons, st.bface, 0.0)
            sim.step(steps)
            cons, bface, _ = sim.get_state(0)
            return (cons, bface), sim.counters(0)
    return with_variant(variant, go)


def drift(cons0, cons1):
    """|sum q(t) - sum q(0)| / sum |q(0)| of the mass, momentum and energy
    totals (exact sums): conservation of a periodic box.  A momentum
    component is measured against the L1 norm of the momentum vector (the
    sum over its three components), so that a component whose total starts
    at or near zero is not divided by its own small norm."""
    import math
    import numpy as np
    norms = [float(np.sum(np.abs(a))) for a in cons0]
    msum = norms[1] + norms[2] + norms[3]
    dens = [norms[0], msum, msum, msum, norms[4]]
    out = {}
    for name, a, b, den in zip(("mass", "mx", "my", "mz", "energy"), cons0, cons1, dens):
        out[name] = float(abs(math.fsum(b.ravel()) - math.fsum(a.ravel())) / (den or 1.0))
    return out


if __name__ == "__main__":
    main()
