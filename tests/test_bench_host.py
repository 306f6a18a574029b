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


def test_flop_counts():
    # plain MR: n_mr (D_Lambda + MR vector work) + the initial residual copy
    assert bench.half_sweep_flops_per_site(4, False) == 4 * (1824 + 336) + 24
    # even/odd: the Schur complement touches every block site once per step, vector work on
    # the even half, one more block sweep for the source and the odd half
    assert bench.half_sweep_flops_per_site(4, True) == 4 * (1824 + 168) + 1824 + 24
    assert bench.sap_flops_per_site(5, 4, True) == 5 * bench.half_sweep_flops_per_site(4, True) + 4.5 * 336
    # one iteration, one cycle: preconditioner + scalings, chi = D phi, GS with k = 0, x update, true residual
    V = 10
    one = (bench.sap_flops_per_site(5, 4) + 48 + 1824 + 144 + 168 + 96 + 1824 + 72) * V
    assert bench.solve_flops(V, 1, 1, 16, 5, 4) == pytest.approx(one)
    # iterations spread over restarts: the second cycle restarts the Gram-Schmidt count
    two_cycles = bench.solve_flops(V, 4, 2, 2, 5, 4)
    assert two_cycles == pytest.approx(2 * bench.solve_flops(V, 2, 1, 2, 5, 4))


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
                        str(tmp_path / "profiles" / "traffic_16c32.json"))
    assert bench.measured_traffic("k_x") == pytest.approx(5.0 * 1024)
    assert bench.measured_traffic("k_missing") is None
    (src / "k.hip").write_text("kernel source, changed\n")
    assert bench.measured_traffic("k_x") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_profile_report(tmp_path):
    """The profile summary: kernel statistics, last-20-dispatch averages beside the bench
    figures, the traffic table per site, and every command that made it."""
    stats = tmp_path / "stats"
    stats.mkdir()
    k = "void wc::k_sap_eo<1, 1, true>(wc::SapLaunch)"
    with open(stats / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "AverageNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": k, "Calls": 25, "AverageNs": 50000.0, "Percentage": 70.0})
    with open(stats / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        # two solves (|b|^2, three half-sweeps, 1 us apart), then 5 warm-up dispatches of
        # 90 us and 20 of 47 us of the timing loop
        for t0 in (0, 50 * 10 ** 6):
            w.writerow({"Kernel_Name": "wc::k_norm2(wc::VecLaunch)", "Start_Timestamp": t0,
                        "End_Timestamp": t0 + 10000})
            for j in range(3):
                w.writerow({"Kernel_Name": k, "Start_Timestamp": t0 + 11000 + j * 48000,
                            "End_Timestamp": t0 + 11000 + j * 48000 + 47000})
        for i in range(25):
            t0 = 100 * 10 ** 6 + i * 10 ** 6
            w.writerow({"Kernel_Name": k, "Start_Timestamp": t0, "End_Timestamp": t0 + (90000 if i < 5 else 47000)})
    rec = {"metric": "m", "roofline": {"launch_ms": 0.0475, "plain_mr_half_sweep_ms": 0.036},
           "dirac": {p: {"ms": 0.02} for p in ("f64", "f32", "f16", "bf16")}}
    (tmp_path / "prof.log").write_text("noise\n" + json.dumps(rec) + "\n")
    (tmp_path / "bench.json").write_text(json.dumps(rec) + "\n")
    traffic = {"fetch_scale": 2.0, "write_scale": 1.0,
               "kernels": {"k_sap_eo<1, 1, true>": {"fetch_bytes": 131072 * 638.0, "write_bytes": 131072 * 144.0}}}
    (tmp_path / "t.json").write_text(json.dumps(traffic))
    out = tmp_path / "r.md"
    bench.profile_report(str(stats), str(tmp_path / "prof.log"), str(tmp_path / "bench.json"),
                         "pf/f_counter_collection.csv", "pw/w_counter_collection.csv", str(tmp_path / "t.json"),
                         str(out))
    md = out.read_text()
    assert f"| `{k}` | 25 | 50.00 | 70.0 |" in md
    assert "(dominant kernel, 4 steps) | 47.00 | 47.50 |" in md
    assert "| `k_sap_eo<1, 1, true>` (one colour) | 638 | 144 |" in md
    assert "rocprofv3 --pmc FETCH_SIZE --output-format csv -d pf -o f -- python -u bench.py --profile" in md
    assert "rocprofv3 --pmc WRITE_SIZE --output-format csv -d pw -o w -- " in md
    assert f"python bench.py --profile-report {stats} " in md
    # the second solve: 4 kernels, 0.151 ms of kernels in a 0.154 ms span
    assert "4 kernels,\n0.15 ms of kernels in a 0.15 ms span" in md
    assert "| `k_sap_eo<1, 1, true>` | 0.141 |" in md
