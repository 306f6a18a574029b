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
