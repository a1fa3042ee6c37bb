"""Host-side logic of bench.py (no GPU): launch-variant parsing, the
kernel names and launch keys that tie rocprofv3 records to launches, the
roofline fractions, and the ingestion of counter records."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_parse_variant_four_or_five_entries():
    assert bench.parse_variant("1,9,64,0") == [1, 9, 64, 0, 64]
    assert bench.parse_variant("3,8,64,1,128") == [3, 8, 64, 1, 128]
    with pytest.raises(SystemExit):
        bench.parse_variant("1,2,3")


def test_kernel_names_and_launch_keys():
    v = [1, 9, 64, 0, 128]
    assert bench.kernel_name("sweep_x", "double", v) == "mhd::k_sweep_x<double, 1, 0, 0>"
    # the y march has no LDS ring: variants 8, 9, 10 run as 2, 6, 7 there
    assert bench.kernel_name("sweep_y", "float", v) == \
        "mhd::k_sweep_march<float, 1, 1, 0, 1, 0, 0, 0, 0>"
    assert bench.kernel_name("sweep_z", "float", v) == \
        "mhd::k_sweep_march<float, 2, 1, 0, 1, 1, 0, 0, 0>"
    assert bench.kernel_name("ct_edge", "double", v) == "mhd::k_ct_edge<double, 0>"
    assert bench.kind_of("void mhd::k_ct_edge<float, 0>(mhd::Launch)") == ("mixed", "ct_edge")
    assert bench.launch_key("sweep_y", "float", v).endswith("|seg=64|persistent=0")
    assert bench.launch_key("sweep_z", "float", v).endswith("|seg=128|persistent=0")
    assert bench.launch_key("sweep_x", "double", v) == "mhd::k_sweep_x<double, 1, 0, 0>|persistent=0"
    for name, want in (("void mhd::k_sweep_x<double, 3, 0, 0>(mhd::Launch)", ("fp64", "sweep_x")),
                       ("void mhd::k_sweep_march<float, 2, 1, 0, 0, 1, 0, 0, 0>(mhd::Launch)",
                        ("mixed", "sweep_z")),
                       ("void mhd::k_ct_face<float>(mhd::Launch)", ("mixed", "ct_face")),
                       ("__amd_rocclr_copyBuffer", None)):
        assert bench.kind_of(name) == want


def test_fused_variants_name_the_xy_march_and_drop_the_x_sweep():
    # x variant 0: window in registers; 2 (mixed path): window in LDS; the
    # march variant then names the z march alone
    for x, real, tail in ((0, "double", "0, 0, 512"), (0, "float", "0, 0, 512"),
                          (2, "float", "1, 0, 256")):
        v = [x, 9, 64, 0, 128]
        name = bench.kernel_name("sweep_y", real, v)
        assert name == f"mhd::k_sweep_march_xy<{real}, {tail}>"
        assert bench.kind_of(f"void {name}(mhd::Launch)")[1] == "sweep_y"
        assert bench.kernel_name("sweep_z", real, v) == \
            f"mhd::k_sweep_march<{real}, 2, 1, 0, 1, 1, 0, 0, 0>"
        prec = 0 if real == "double" else 1
        t = bench.bytes_table(prec, v)
        assert "sweep_x" not in t and t["sweep_y"][0] > bench.bytes_table(prec, [1] + v[1:])["sweep_y"][0]


def test_fractions_arithmetic():
    cells = 1000
    table = {"a": (100, 100), "b": (50, 70)}
    f = bench.fractions(1.0, cells, table, 1e12, triad_gbs=4000.0)
    nbytes = (200 + 120) * cells
    assert f["design_hbm"] == round(nbytes / (bench.HBM_PEAK_GBS * 1e9) / 1e-3, 4)
    assert f["design_vs_measured_triad"] == round(nbytes / 4e12 / 1e-3, 4)
    assert "design_vs_measured_triad" not in bench.fractions(1.0, cells, table, 1e12)


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                           "Counter_Value"])
        w.writeheader()
        for i, (k, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": k, "Counter_Name": counter,
                        "Counter_Value": v})


def test_byte_tables_sum_to_the_step_totals():
    """Per cell-update (one SSP-RK2 step, both stages) the algorithmic bytes
    of the kernels add up to the design's totals: 1424 B FP64 and 1024 B
    mixed with the x sweep, 1136 B and 816 B with the fused march (which
    replaces the x sweep and the y march)."""
    def total(t):
        return sum(a + b for a, b in t.values())
    assert total(bench.bytes_table(0, [1, 1, 64, 0, 64])) == 1424
    assert total(bench.bytes_table(1, [1, 1, 64, 0, 128])) == 1024
    assert total(bench.bytes_table(0, [0, 1, 64, 0, 64])) == 1136
    assert total(bench.bytes_table(1, [2, 9, 64, 0, 128])) == 816
    for p in (0, 1):
        assert "sweep_x" not in bench.bytes_table(p, [0, 1, 64, 0, 64])


def test_roofline_of_the_dominant_kernel(monkeypatch):
    """The dominant kernel is the one with the largest time per step
    (average launch time x launches); its bytes per launch are the mean of
    the stages' algorithmic bytes (first stage once, later stages rk - 1
    times); achieved = bytes / average launch time; traffic and VALU issue
    come from the committed records when they match, else null."""
    cells = 1_000_000
    table = {"sweep_y": (176, 176), "sweep_z": (168, 208), "ct_edge": (120, 120)}
    kt = {"sweep_y": (8.0, 20), "sweep_z": (5.0, 20), "ct_edge": (9.0, 10)}
    monkeypatch.setattr(bench, "recorded_kernel", lambda path, p, dom, v: None)
    a = bench.argparse.Namespace(workload="turbulence", n=100)
    r = bench.roofline(kt, cells, table, [0, 1, 64, 0, 64], 0, a)
    assert r["kernel"] == "sweep_y" and r["bytes_per_launch"] == 176 * cells
    assert r["achieved"] == round(176 * cells / 8e-3 / 1e9, 1)
    assert r["frac"] == round(r["achieved"] / 8000.0, 4) and r["traffic"] is None
    kt = {"sweep_y": (4.0, 20), "sweep_z": (5.0, 20), "ct_edge": (1.0, 20)}
    r = bench.roofline(kt, cells, table, [0, 1, 64, 0, 64], 0, a, rk=3)
    assert r["kernel"] == "sweep_z"
    assert r["bytes_per_launch"] == int((168 + 2 * 208) / 3 * cells)
    rec = {"bytes": 9_000_000_000, "valu_issue": 0.5, "valu_per_wave": 100.0}
    monkeypatch.setattr(bench, "recorded_kernel", lambda path, p, dom, v: rec)
    r = bench.roofline(kt, cells, table, [0, 1, 64, 0, 64], 0, a, rk=3)
    assert r["traffic"] == 9_000_000_000 and r["valu_issue"] == 0.5
    assert r["traffic_over_algorithmic"] == round(9e9 / ((168 + 2 * 208) / 3 * cells), 3)


def test_ingest_counters_scales_by_the_calibration_copy(tmp_path, monkeypatch):
    """FETCH_SIZE reads half the copy's bytes and WRITE_SIZE all of them in
    this synthetic record: the scales are 2 and 1, and each kernel's traffic
    is its averaged readings times those scales."""
    kib = bench.COPY_BYTES / 1024
    x64 = "void mhd::k_sweep_x<double, 1, 0, 0>(mhd::Launch)"
    fetch = [("__amd_rocclr_copyBuffer", kib / 2)] * 3 + [(x64, 1000.0), (x64, 1200.0)]
    write = [("__amd_rocclr_copyBuffer", kib)] * 3 + [(x64, 500.0), (x64, 700.0)]
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(f, "FETCH_SIZE", fetch)
    _counter_csv(w, "WRITE_SIZE", write)
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "profile_file", lambda kind, a, ext: str(out))
    args = bench.argparse.Namespace(ingest_counters=(str(f), str(w)), n=8, fetch_command="f",
                                    write_command="w", variant64="1,2,64,0,64",
                                    variant_mixed="1,8,64,0,128", workload="blast")
    bench.ingest_counters(args)
    rec = json.loads(out.read_text())
    assert rec["scale"] == {"fetch": 2.0, "write": 1.0}
    k = rec["fp64"]["kernels"]["sweep_x"]
    assert k["dispatches"] == 2 and k["fetch_kib"] == 1100.0 and k["write_kib"] == 600.0
    assert k["bytes"] == int((1100.0 * 2.0 + 600.0) * 1024)
    assert k["launch"] == bench.launch_key("sweep_x", "double", [1, 2, 64, 0, 64])


def test_ingest_waves_divides_each_counter_by_the_wave_cycles(tmp_path, monkeypatch):
    """Each counter is summed over the kernel's dispatches and divided by the
    summed wave-cycles; kernels outside the benchmark's kinds and counters
    outside the pass are ignored."""
    xy = "void mhd::k_sweep_march_xy<double, 0, 0, 512>(mhd::Launch)"
    rows = []
    for i, (cyc, valu, wait) in enumerate(((1000.0, 300.0, 400.0), (3000.0, 900.0, 1200.0))):
        for c, v in (("SQ_WAVE_CYCLES", cyc), ("SQ_ACTIVE_INST_VALU", valu), ("SQ_WAIT_ANY", wait),
                     ("SQ_WAIT_INST_ANY", cyc / 5), ("SQ_ACTIVE_INST_LDS", cyc / 100),
                     ("SQ_WAIT_INST_LDS", 0.0), ("SQ_BUSY_CYCLES", 7.0)):
            rows.append({"Dispatch_Id": i, "Kernel_Name": xy, "Counter_Name": c,
                         "Counter_Value": v})
    rows.append({"Dispatch_Id": 9, "Kernel_Name": "__amd_rocclr_copyBuffer",
                 "Counter_Name": "SQ_WAVE_CYCLES", "Counter_Value": 5.0})
    path = tmp_path / "w.csv"
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)
    monkeypatch.setattr(bench, "profile_file",
                        lambda kind, a, ext: str(tmp_path / f"{kind}.{ext}"))
    args = bench.argparse.Namespace(ingest_waves=str(path), n=512, workload="turbulence",
                                    waves_command="cmd", variant64="0,1,64,0,64",
                                    variant_mixed="0,9,128,0,128")
    bench.ingest_waves(args)
    rec = json.loads((tmp_path / "sq_wave_cycles.json").read_text())
    assert list(rec["fp64"]) == [xy] and rec["mixed"] == {}
    f = rec["fp64"][xy]
    assert f == {"SQ_ACTIVE_INST_VALU": 0.3, "SQ_WAIT_ANY": 0.4, "SQ_WAIT_INST_ANY": 0.2,
                 "SQ_ACTIVE_INST_LDS": 0.01, "SQ_WAIT_INST_LDS": 0.0}
    md = (tmp_path / "sq_wave_cycles.md").read_text()
    assert "| fp64 | `mhd::k_sweep_march_xy<double, 0, 0, 512>` | 0.30 | 0.40 | 0.20 | 0.01 | 0.00 |" in md
    assert "cmd" in md


def test_ingest_sq_issue_rate_and_record(tmp_path, monkeypatch):
    """VALU issue is the mean VALU instructions per dispatch over the mean
    traced duration times the chip's issue ceiling (1024 SIMDs at 2.4 GHz,
    4 cycles per wave64 instruction); per-wave figures divide by the mean
    wave count; the record is keyed by the launch the variant names."""
    xy = "void mhd::k_sweep_march_xy<double, 0, 0, 512>(mhd::Launch)"
    valu = 0.5 * 2e-3 * bench.VALU_ISSUE_PER_S  # half the slots over 2 ms
    rows = []
    for i in range(2):
        for c, v in (("SQ_WAVES", 32768.0), ("SQ_INSTS_VALU", valu), ("SQ_INSTS_SALU", 3276.8),
                     ("SQ_INSTS_VMEM_RD", 65536.0), ("SQ_INSTS_LDS", 1000.0),
                     ("SQ_LDS_BANK_CONFLICT", 250.0)):
            rows.append({"Dispatch_Id": i, "Kernel_Name": xy, "Counter_Name": c,
                         "Counter_Value": v})
    sq = tmp_path / "sq.csv"
    with open(sq, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)
    tdir = tmp_path / "trace"
    tdir.mkdir()
    with open(tdir / "run_kernel_trace.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp",
                                           "VGPR_Count", "SGPR_Count", "LDS_Block_Size",
                                           "Scratch_Size"])
        w.writeheader()
        for start, end in ((0, 1_000_000), (5_000_000, 8_000_000)):  # 1 ms and 3 ms
            w.writerow({"Kernel_Name": xy, "Start_Timestamp": start, "End_Timestamp": end,
                        "VGPR_Count": 128, "SGPR_Count": 112, "LDS_Block_Size": 127488,
                        "Scratch_Size": 16})
    monkeypatch.setattr(bench, "profile_file",
                        lambda kind, a, ext: str(tmp_path / f"{kind}.{ext}"))
    args = bench.argparse.Namespace(ingest_sq=(str(sq), str(tdir)), n=512, workload="turbulence",
                                    sq_command="sq", trace_command="kt",
                                    variant64="0,1,64,0,64", variant_mixed="0,9,128,0,128")
    bench.ingest_sq(args)
    rec = json.loads((tmp_path / "sq_counters.json").read_text())
    k = rec["fp64"]["kernels"]["sweep_y"]
    assert k["launch"] == bench.launch_key("sweep_y", "double", [0, 1, 64, 0, 64])
    assert k["valu_issue"] == 0.5 and k["avg_us_unfused"] == 2000.0
    assert k["valu_per_wave"] == round(valu / 32768, 1)
    assert k["lds_conflict_per_instr"] == 0.25 and k["scratch_bytes"] == "16"
    md = (tmp_path / "sq_counters.md").read_text()
    assert "| fp64 | `mhd::k_sweep_march_xy<double, 0, 0, 512>` | 32768 |" in md


def test_summarize_trace_matches_the_bench_launch_shape(tmp_path, monkeypatch):
    """The agreement row of each precision averages the dominant kernel's
    dispatches of the launch shape with the most dispatches (the timed run,
    not the autotuner's trial shapes) and divides by the bench's HIP-event
    average."""
    xy64 = "void mhd::k_sweep_march_xy<double, 0, 0, 512>(mhd::Launch)"
    xy32 = "void mhd::k_sweep_march_xy<float, 0, 0, 512>(mhd::Launch)"
    tdir = tmp_path / "kt"
    tdir.mkdir()
    with open(tdir / "run_kernel_stats.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "AverageNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": xy64, "Calls": 8, "AverageNs": 8.0e6, "Percentage": 60.0})
        w.writerow({"Name": xy32, "Calls": 4, "AverageNs": 6.0e6, "Percentage": 40.0})
    with open(tdir / "run_kernel_trace.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size_X", "Start_Timestamp",
                                           "End_Timestamp"])
        w.writeheader()
        t = 0
        for name, grid, us in ([(xy64, 2097152, 8600)] * 6 + [(xy64, 1048576, 3000)] * 2
                               + [(xy32, 1048576, 6000)] * 4):
            w.writerow({"Kernel_Name": name, "Grid_Size_X": grid, "Start_Timestamp": t,
                        "End_Timestamp": t + us * 1000})
            t += us * 1000 + 10
    line = {"metric": "m", "value": 3400.0, "source_sha": "abc",
            "config": {"variant": [0, 1, 64, 0, 64]},
            "roofline": {"kernel": "sweep_y", "avg_launch_ms": 8.6},
            "mixed": {"value": 4900.0, "variant": [0, 9, 128, 0, 128],
                      "roofline": {"kernel": "sweep_y", "avg_launch_ms": 5.0}}}
    log = tmp_path / "bench.log"
    log.write_text("noise\n" + json.dumps(line) + "\n")
    monkeypatch.setattr(bench, "profile_file",
                        lambda kind, a, ext: str(tmp_path / f"{kind}.{ext}"))
    args = bench.argparse.Namespace(summarize_trace=(str(tdir), str(log)), n=512,
                                    workload="turbulence", trace_command="kt")
    bench.summarize_trace(args)
    md = (tmp_path / "kernel_trace.md").read_text()
    assert "| fp64 | `mhd::k_sweep_march_xy<double, 0, 0, 512>` | 2097152 | 6 | 8600.0 | 8600.0 | 1.000 |" in md
    assert "| mixed | `mhd::k_sweep_march_xy<float, 0, 0, 512>` | 1048576 | 4 | 6000.0 | 5000.0 | 1.200 |" in md
    assert "Kernel source hash abc" in md


def test_counter_records_take_the_variants_of_their_commands(monkeypatch):
    """Ingestion keys a counter record by the launch variants the recorded
    counter runs used, unless they are given explicitly."""
    cmd = ("rocprofv3 --pmc FETCH_SIZE -f csv -d out -o run -- python -u bench.py --counter-pass "
           "--steps 2 --variant64 1,2,64,0,64 --variant-mixed 1,8,64,0,128")
    assert bench.variant_in_command(cmd, "--variant-mixed") == "1,8,64,0,128"
    assert bench.variant_in_command("python bench.py", "--variant64") is None
    monkeypatch.setattr(sys, "argv", ["bench.py", "--ingest-counters", "f.csv", "w.csv",
                                      "--fetch-command", cmd])
    a = bench.parse()
    assert (a.variant64, a.variant_mixed) == ("1,2,64,0,64", "1,8,64,0,128")
    monkeypatch.setattr(sys, "argv", ["bench.py", "--ingest-counters", "f.csv", "w.csv",
                                      "--fetch-command", cmd, "--variant64", "3,9,16,1,32"])
    assert bench.parse().variant64 == "3,9,16,1,32"
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    fixed = bench.BENCH_VARIANTS[("turbulence", 512)]
    assert (a.workload, a.n, a.fixed_steps) == ("turbulence", 512, 200)
    assert (a.variant64, a.variant_mixed) == (fixed["fp64"], fixed["mixed"])
    monkeypatch.setattr(sys, "argv", ["bench.py", "--workload", "blast", "--n", "96"])
    a = bench.parse()
    assert (a.n, a.fixed_steps, a.cpu_n) == (96, 100, 256)
    assert (a.variant64, a.variant_mixed) == ("1,1,64,0,64", "1,1,64,0,128")


def test_recorded_kernel_needs_matching_source_and_variant(tmp_path):
    """A counter record is used only for the kernel source and the launch
    variant it was taken on."""
    v = [1, 2, 64, 0, 64]
    rec = {"source_sha": bench.source_sha(),
           "fp64": {"kernels": {"sweep_x": {"launch": bench.launch_key("sweep_x", "double", v),
                                            "bytes": 123, "valu_issue": 0.5}}}}
    path = tmp_path / "r.json"
    path.write_text(json.dumps(rec))
    assert bench.recorded_kernel(str(path), 0, "sweep_x", v)["bytes"] == 123
    assert bench.recorded_kernel(str(path), 0, "sweep_x", [3, 2, 64, 0, 64]) is None
    assert bench.recorded_kernel(str(path), 1, "sweep_x", v) is None
    rec["source_sha"] = "0" * 16
    path.write_text(json.dumps(rec))
    assert bench.recorded_kernel(str(path), 0, "sweep_x", v) is None


def test_drift_of_totals():
    import numpy as np
    a = [np.array([1.0, 2.0, -3.0])] * 5
    b = [np.array([1.0, 2.0, -3.0 + 6e-12])] * 5
    d = bench.drift(a, b)
    assert set(d) == {"mass", "mx", "my", "mz", "energy"}
    assert abs(d["mass"] - 1e-12) < 1e-15
    # momentum components against the momentum vector's L1 norm (18 here)
    assert abs(d["mz"] - 6e-12 / 18.0) < 1e-15
    # a component that starts at zero is not divided by its own zero norm
    z = [a[0], a[1], a[2], np.zeros(3), a[4]]
    d = bench.drift(z, [a[0], a[1], a[2], np.array([0.0, 0.0, 1.2e-11]), a[4]])
    assert abs(d["mz"] - 1.2e-11 / 12.0) < 1e-15


def test_committed_records_describe_the_benchmark_kernels():
    """The HBM-traffic and SQ-counter records of the benchmark workload were
    taken on the current kernel sources with the launch variants the bench
    runs, so the bench line's roofline carries their traffic and VALU issue
    for the dominant kernel of both precisions.  A kernel change makes them
    stale until the counter runs are repeated (their commands are in the
    records)."""
    a = bench.argparse.Namespace(workload="turbulence", n=512)
    variants = bench.BENCH_VARIANTS[("turbulence", 512)]
    for precision, key in ((0, "fp64"), (1, "mixed")):
        v = bench.parse_variant(variants[key])
        for kind in ("hbm_traffic", "sq_counters"):
            path = bench.profile_file(kind, a, "json")
            assert bench.recorded_kernel(path, precision, "sweep_y", v) is not None, (kind, key)
