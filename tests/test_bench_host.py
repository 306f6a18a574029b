"""Host logic of bench.py (CPU): nominal flop counts, the rocprofv3 counter summary (copy
calibration, the last 20 dispatches of each kernel), the staleness check of the committed
traffic record, and the one-GPU limit."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_flop_and_byte_counts():
    # D_Lambda on 4^4 blocks: 6 of the 8 hops stay in the block (144 flops each), 5
    # accumulates of 24, both clover blocks 504
    assert bench.mean_inblock_hops((4, 4, 4, 4)) == 6.0
    assert bench.dlambda_flops((4, 4, 4, 4)) == 6 * 144 + 5 * 24 + 504 == 1488
    # even/odd half-sweep per solved site: 4 Schur steps (operator + half the MR vector work),
    # one more block sweep for the source and the odd half, 12, the 2 border hops with their
    # accumulates, and psi += z
    assert bench.half_sweep_flops((4, 4, 4, 4), 4, True) == 4 * (1488 + 168) + 1488 + 12 + 2 * 168 + 24 == 8484
    assert bench.half_sweep_flops((4, 4, 4, 4), 4, True, executed=False) == 4 * (1824 + 168) + 1824 + 12 + 336 + 24
    assert bench.half_sweep_flops((4, 4, 4, 4), 4, False) == 4 * (1488 + 336) + 336 + 24
    # bytes: 16-bit operator 148 + 152, six 52-byte spinor passes; D_w FP64 1536 per site
    assert bench.half_sweep_bytes("bf16") == 612
    assert bench.half_sweep_bytes("bf16", tile=12) == pytest.approx(300 / 12 + 312)
    assert bench.dw_bytes("f64") == 1536 and bench.dw_bytes("f32", tile=2) == 192 + 288
    # one FGCR iteration in one cycle: SAP (ncy half-sweeps over half the sites each, counted
    # per site) + scalings, D, Gram-Schmidt with k = 0, then the x update and true residual
    one = (5 * bench.half_sweep_flops((4, 4, 4, 4), 4, True) + 48 + 1824 + 144 + 168 + 96 + 1824 + 72) * 10
    assert bench.solve_flops(10, 1, 1, 16, 5, 4, (4, 4, 4, 4), True) == pytest.approx(one)
    two = bench.solve_flops(10, 4, 2, 2, 5, 4, (4, 4, 4, 4), True)
    assert two == pytest.approx(2 * bench.solve_flops(10, 2, 1, 2, 5, 4, (4, 4, 4, 4), True))


def _pmc_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (kernel, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": kernel, "Counter_Name": counter, "Counter_Value": value})


def test_summarise_pmc_scales_by_the_copy_and_keeps_the_last_20(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    k = "void wc::k_dirac<1, 1, false>(wc::DiracLaunch)"
    # FETCH_SIZE reads half of the 1 GiB copy (factor 2), WRITE_SIZE all of it (factor 1);
    # the first 5 dispatches of the kernel (warm-up) differ from the last 20
    gib_kib = float(1 << 20)
    fetch = [(copy, gib_kib / 2)] + [(k, 999.0)] * 5 + [(k, 100.0)] * 20
    write = [(copy, gib_kib)] + [(k, 777.0)] * 5 + [(k, 10.0)] * 20
    _pmc_csv(tmp_path / "f.csv", "FETCH_SIZE", fetch)
    _pmc_csv(tmp_path / "w.csv", "WRITE_SIZE", write)
    rec = bench.summarise_pmc(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "t.json"))
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    kr = rec["kernels"]["k_dirac<1, 1, false>"]
    assert kr["launches"] == 20
    assert kr["fetch_bytes"] == pytest.approx(2.0 * 100.0 * 1024)
    assert kr["write_bytes"] == pytest.approx(10.0 * 1024)
    assert kr["bytes_per_launch"] == pytest.approx(kr["fetch_bytes"] + kr["write_bytes"])
    assert json.load(open(tmp_path / "t.json"))["kernels"].keys() == {"k_dirac<1, 1, false>"}


def test_traffic_record_is_dropped_when_the_sources_change(tmp_path, monkeypatch):
    src = tmp_path / "paper_1109_4279_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "k.hip").write_text("kernel source\n")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    copy = "__amd_rocclr_copyBuffer"
    k = "void wc::k_x(wc::VecLaunch)"
    _pmc_csv(tmp_path / "f.csv", "FETCH_SIZE", [(copy, float(1 << 20))] + [(k, 4.0)] * 20)
    _pmc_csv(tmp_path / "w.csv", "WRITE_SIZE", [(copy, float(1 << 20))] + [(k, 1.0)] * 20)
    bench.summarise_pmc(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"),
                        str(tmp_path / "profiles" / "traffic_24c48.json"))
    assert bench.measured_traffic("k_x", "traffic_24c48.json") == pytest.approx(5.0 * 1024)
    assert bench.measured_traffic("k_missing", "traffic_24c48.json") is None
    assert bench.measured_traffic("k_x", "missing.json") is None
    (src / "k.hip").write_text("kernel source, changed\n")
    assert bench.measured_traffic("k_x", "traffic_24c48.json") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_profile_summary(tmp_path):
    """The committed profile summary: kernels by total time, the last 20 dispatches' mean
    beside the overall mean, the traffic per launch when a record is given, the command."""
    k = "void wc::k_sap_eo<3, 1, false>(wc::SapLaunch)"
    g = "wc::k_gs_dots(wc::VecLaunch)"
    with open(tmp_path / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": g, "Calls": 2, "TotalDurationNs": 2000.0, "AverageNs": 1000.0, "Percentage": 10.0})
        w.writerow({"Name": k, "Calls": 25, "TotalDurationNs": 25 * 50000.0, "AverageNs": 50000.0,
                    "Percentage": 90.0})
    with open(tmp_path / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for i in range(25):
            t0 = i * 10 ** 6
            w.writerow({"Kernel_Name": k, "Start_Timestamp": t0, "End_Timestamp": t0 + (90000 if i < 5 else 40000)})
        for i in range(2):
            w.writerow({"Kernel_Name": g, "Start_Timestamp": 10 ** 9 + i, "End_Timestamp": 10 ** 9 + i + 1000})
    (tmp_path / "t.json").write_text(json.dumps({"kernels": {"k_sap_eo<3, 1, false>": {"bytes_per_launch": 2.5e9}}}))
    lines = bench.profile_summary(str(tmp_path), str(tmp_path / "o.md"), "rocprofv3 ... -- python3 bench.py --profile",
                                  str(tmp_path / "t.json"))
    md = (tmp_path / "o.md").read_text()
    assert md.startswith("Command: `rocprofv3 ... -- python3 bench.py --profile`")
    assert lines[4] == "| `k_sap_eo<3, 1, false>` | 25 | 50.00 | 40.00 | 1.250 | 90.0 | 2500.0 |"
    assert lines[5] == "| `k_gs_dots` | 2 | 1.00 | 1.00 | 0.002 | 10.0 |  |"


def test_counter_summary(tmp_path):
    """Per-counter means over the last dispatches of the matching kernels."""
    rows = []
    for i in range(25):
        rows.append(("void wc::k_sap_eo<3, 1, false>(wc::SapLaunch)", "SQ_INSTS_VALU", 100.0 if i < 5 else 10.0))
        rows.append(("void wc::k_sap_eo<3, 1, false>(wc::SapLaunch)", "GRBM_GUI_ACTIVE", 7.0))
        rows.append(("wc::k_gs_dots(wc::VecLaunch)", "SQ_INSTS_VALU", 1.0))
    with open(tmp_path / "c.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (k, c, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})
    rec = bench.counter_summary(str(tmp_path / "c.csv"), str(tmp_path / "c.md"), "cmd")
    assert rec == {"k_sap_eo<3, 1, false>": {"SQ_INSTS_VALU": 10.0, "GRBM_GUI_ACTIVE": 7.0}}
    md = (tmp_path / "c.md").read_text()
    assert "| `k_sap_eo<3, 1, false>` | 7 | 10 |" in md


def test_valu_record(tmp_path, monkeypatch):
    """VALU occupancy: 4 cycles per wave64 instruction over SIMDs and per-XCD cycles, for the
    launches with MR steps (the last 20), those without (the 20 before that differ) and
    their difference; dropped once the kernel sources change."""
    src = tmp_path / "paper_1109_4279_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "k.hip").write_text("kernel source\n")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    k = "void wc::k_sap_eo<3, 1, false>(wc::SapLaunch)"
    rows = []
    # 22 launches without MR steps: 100 instructions, 800 GRBM cycles (100 per XCD);
    # then 22 with: 300 instructions, 1600 cycles (200 per XCD)
    for i in range(44):
        v, g = (100.0, 800.0) if i < 22 else (300.0, 1600.0)
        rows += [(i, k, "SQ_INSTS_VALU", v), (i, k, "GRBM_GUI_ACTIVE", g)]
    with open(tmp_path / "q.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, kk, c, v in rows:
            w.writerow({"Dispatch_Id": i, "Kernel_Name": kk, "Counter_Name": c, "Counter_Value": v})
    out = tmp_path / "profiles" / "valu_24c48.json"
    bench.valu_record(str(tmp_path / "q.csv"), str(out), simds=4, xcds=8)
    r = bench.measured_valu("k_sap_eo<3, 1, false>", "valu_24c48.json")
    assert r["valu_busy_launch"] == pytest.approx(300 * 4 / (4 * 200))
    assert r["valu_busy_without_mr_steps"] == pytest.approx(100 * 4 / (4 * 100))
    assert r["valu_busy_mr_steps"] == pytest.approx(200 * 4 / (4 * 100))
    (src / "k.hip").write_text("changed\n")
    assert bench.measured_valu("k_sap_eo<3, 1, false>", "valu_24c48.json") is None
