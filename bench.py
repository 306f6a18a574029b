"""Benchmark of the Wilson-clover SAP-FGCR hot path on one MI355X.

One step = one complete mixed-precision solve D x = b to a true FP64 residual of 1e-10
(FP32 Schwarz preconditioner on FP32 storage, FP64 outer FGCR) on the 16^3 x 32 lattice
(gauge recipe eps = 0.3, m0 = -0.1, c_sw = 1, 4^4 Schwarz blocks, 4 MR steps of the
even/odd-preconditioned block solver, 5 SAP cycles, restart 16, one Gaussian source),
inputs resident on the device.

`value` is the sustained solver throughput in Gflop/s (nominal flops of every kernel of
the solve divided by the step time).  Beside it: the FP64 solve time on the same system
(with the same block solver and with MR on the unpreconditioned block operator), the
mixed solve with the unpreconditioned block solver, D_w GB/s and Gflop/s per storage
precision against the 8 TB/s HBM roofline, the roofline record of the dominant kernel
(the Schwarz block solver against the vector-ALU peak, with its two phases: the set-up that
moves the operator and the fields, and the MR steps that run from registers and LDS),
the batched 12-point-source solve on
24^3 x 48 against 12 single FP64 solves, the 32^3 x 64 solve on 16-bit storage, FGCR
against FGMRES-DR close to the critical mass (the regime of the paper's Fig. 1), and the
FP64 oracle timed on the host for a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DIMS = (32, 16, 16, 16)
BLOCK = (4, 4, 4, 4)
M0, CSW = -0.1, 1.0
NKV, NCY, NMR, TOL = 16, 5, 4, 1e-10
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# FP32 FMA rate of the kernels as built (no packed FP32 instructions): 256 CUs x 4 SIMDs
# x 16 lanes x 2 flop x 2.4 GHz
FP32_SCALAR_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

# algorithmic bytes per site of one D_w application: spinor in + out, 4 links, 2 clover blocks
DW_BYTES = {"f64": 192 + 192 + 576 + 576, "f32": 96 + 96 + 288 + 288, "f16": 52 + 52 + 148 + 152,
            "bf16": 52 + 52 + 148 + 152}
DW_FLOPS = 1320 + 504
# Schwarz half-sweep, per solved site (FP32 storage): links + clover of the block, residual in and
# out, block solution out, psi in and out, and the neighbouring blocks' solution read once
SAP_BYTES_F32 = 288 + 288 + 96 * 2 + 96 + 96 * 2 + 96
MR_VEC_FLOPS = 336          # per site and MR step: <q,rho>, <q,q>, z += a rho, rho -= a q
BORDER_FLOPS_4444 = 2 * 168  # 2 cross-block hops per site on 4^4 blocks (project + SU(3) + add)


def half_sweep_flops_per_site(nmr, eo):
    """Nominal flops of one Schwarz half-sweep per solved site, D_Lambda counted as the full
    1824 flops of D_w.  Plain block solver: nmr MR steps on D_Lambda.  Even/odd block solver:
    an application of the Schur complement touches every site of the block once (hops and a
    6x6 clover pair), the MR vector work runs on the even half, and the source (A_oo^-1,
    H_eo) and the odd half of the solution (H_oe, A_oo^-1) add one more block sweep."""
    if eo:
        return nmr * (DW_FLOPS + MR_VEC_FLOPS / 2) + DW_FLOPS + 24
    return nmr * (DW_FLOPS + MR_VEC_FLOPS) + 24


def sap_flops_per_site(ncy, nmr, eo=False):
    """Nominal flops of one SAP application per lattice site."""
    return ncy * half_sweep_flops_per_site(nmr, eo) + (ncy - 0.5) * BORDER_FLOPS_4444


def solve_flops(V, iters, restarts, nkv, ncy, nmr, eo=False):
    """Nominal flops of a restarted SAP-FGCR solve with `iters` iterations over `restarts` cycles."""
    f = 0.0
    left = iters
    for _ in range(max(restarts, 1)):
        kd = min(nkv, left)
        left -= kd
        for k in range(kd):
            f += sap_flops_per_site(ncy, nmr, eo) + 48   # preconditioner + scaling in/out
            f += DW_FLOPS                                  # chi = D phi (FP64)
            f += 2 * 96 * k + 144 + 168                     # CGS dots + update, norms, r update
        f += 96 * kd + DW_FLOPS + 72                        # x update, true residual
    return f * V


def cpu_baseline(U, b):
    """The FP64 oracle on a bounded sample of the same workload: one FGCR iteration
    (one SAP application with 4 even/odd block-solver steps x 5 cycles, chi = D phi,
    Gram-Schmidt) on the 16^3 x 32 system, single thread, reported in the same Gflop/s unit."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import dirac, solvers

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        A = dirac.clover_matrix(U, M0, CSW)
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        res = solvers.fgcr(lambda v: dirac.apply_D(U, A, v),
                           lambda v: solvers.sap(U, A, v, BLOCK, NMR, NCY, eo=True),
                           b, tol=1e-300, nkv=NKV, maxit=1)
        t = time.perf_counter() - t0
    V = int(np.prod(DIMS))
    fl = solve_flops(V, 1, 1, NKV, NCY, NMR, eo=True)
    return {"value": fl / t / 1e9, "unit": "Gflop/s", "cores": 1, "kind": "oracle",
            "sample": f"one FGCR iteration (SAP {NCY} cycles x {NMR} even/odd block-solver steps + FP64 D + GS + "
                      f"true residual) of the 16^3x32 workload, numpy FP64, 1 thread; {t:.1f} s (clover setup "
                      f"{t_setup:.1f} s not counted)",
            "seconds": t, "iters_done": res.iters}


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    runs (profiles/traffic_16c32.json), or None when the kernel sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_16c32.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    src = os.path.join(ROOT, "paper_1109_4279_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(src)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(src, f), "rb").read())
    if rec.get("csrc_sha256") != h.hexdigest() or kernel not in rec.get("kernels", {}):
        return None
    return rec["kernels"][kernel]["bytes_per_launch"]


def timed_solve(lat, b, params, torch):
    lat.solve(b, params)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, st = lat.solve(b, params)
    torch.cuda.synchronize()
    return x, st, (time.perf_counter() - t0) * 1e3


def params(wc, sap_prec, eo):
    return wc.default_params(nkv=NKV, ncy=NCY, nmr=NMR, tol=TOL, sap_prec=sap_prec, eo=int(eo), use_graph=1)


def single_solves(lat, srcs, p, torch):
    """Mean time per rhs of solving the sources one at a time (after a warm-up solve)."""
    lat.solve(srcs[0].contiguous(), p)
    torch.cuda.synchronize()
    t, iters = 0.0, []
    for r in range(srcs.shape[0]):
        src = srcs[r].contiguous()
        t0 = time.perf_counter()
        _, st1 = lat.solve(src, p)
        torch.cuda.synchronize()
        t += (time.perf_counter() - t0) * 1e3 / srcs.shape[0]
        iters.append(st1[0]["iters"])
    return t, max(iters)


def extra_workloads(wc, torch, dev):
    """Batched 12-point-source solve on 24^3 x 48 (FP32 arithmetic on FP16 storage, even/odd
    block solver) against 12 single FP64 solves (with MR on D_Lambda, the plain method, and
    with the same block solver), and the 32^3 x 64 single-rhs solve on every storage."""
    import synth
    out = {}
    dims = (48, 24, 24, 24)
    lat = wc.Lattice(torch.from_numpy(synth.gauge_field(dims)).to(dev), block=BLOCK, m0=M0, csw=CSW)
    pts = torch.from_numpy(synth.point_sources(dims)).to(dev)
    t_mr, it_mr = single_solves(lat, pts, params(wc, "f64", False), torch)
    t_eo, it_eo = single_solves(lat, pts, params(wc, "f64", True), torch)
    xb, stb, t_batch = timed_solve(lat, pts, params(wc, "f16", True), torch)
    res = max(s["rel_true_res"] for s in stb)
    out["batch_24c48_12rhs"] = {
        "fp64_single_rhs_ms": t_mr, "fp64_single_rhs_iters": it_mr,
        "fp64_eo_single_rhs_ms": t_eo, "fp64_eo_single_rhs_iters": it_eo,
        "mixed_f16_eo_batched_12rhs_ms": t_batch, "iters_batched": max(s["iters"] for s in stb),
        "speedup_per_rhs": 12 * t_mr / t_batch, "speedup_per_rhs_vs_fp64_eo": 12 * t_eo / t_batch,
        "max_true_rel_residual": res, "target": 3.0}
    del lat, pts, xb
    dims = (64, 32, 32, 32)
    lat = wc.Lattice(torch.from_numpy(synth.gauge_field(dims)).to(dev), block=BLOCK, m0=M0, csw=CSW)
    b = torch.from_numpy(synth.gaussian_spinor(dims)).to(dev)
    rec = {}
    _, st_mr, t_mr = timed_solve(lat, b, params(wc, "f64", False), torch)
    rec["fp64_mr_ms"], rec["fp64_mr_iters"] = t_mr, st_mr[0]["iters"]
    x64, st64, t64 = timed_solve(lat, b, params(wc, "f64", True), torch)
    rec["fp64_ms"], rec["fp64_iters"] = t64, st64[0]["iters"]
    for sp in ("f32", "f16", "bf16"):
        x, st, t = timed_solve(lat, b, params(wc, sp, True), torch)
        rel = (torch.linalg.vector_norm(x - x64) / torch.linalg.vector_norm(x64)).item()
        rec[sp] = {"ms": t, "iters": st[0]["iters"], "true_rel_residual": st[0]["rel_true_res"],
                   "rel_err_vs_fp64_solution": rel}
    out["solve_32c64"] = rec
    del lat, b
    out["near_critical_16c32"] = near_critical(wc, torch, dev)
    return out


def near_critical(wc, torch, dev):
    """The regime of the paper's Fig. 1: m0 = -0.178, close to the critical mass of the
    synthetic eps = 0.3 field on 16^3 x 32.  FGCR with restart 16 and 32 against
    FGMRES-DR with 32 vectors of which 10 are deflated harmonic Ritz vectors; same FP32
    even/odd SAP preconditioner, FP64 outer solver, tol 1e-10."""
    import synth
    m0 = -0.178
    lat = wc.Lattice(torch.from_numpy(synth.gauge_field(DIMS)).to(dev), block=BLOCK, m0=m0, csw=CSW)
    b = torch.from_numpy(synth.gaussian_spinor(DIMS)).to(dev)
    rec = {"m0": m0}

    def run(name, f):
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = f()
        torch.cuda.synchronize()
        rec[name] = {"ms": (time.perf_counter() - t0) * 1e3, "iters": st[0]["iters"],
                     "restarts": st[0]["restarts"], "true_rel_residual": st[0]["rel_true_res"],
                     "status": st[0]["status"]}

    kw = dict(ncy=NCY, nmr=NMR, tol=TOL, sap_prec="f32", eo=1, maxit=3000)
    run("fgcr_16", lambda: lat.solve(b, check=False, nkv=16, **kw))
    run("fgcr_32", lambda: lat.solve(b, check=False, nkv=32, **kw))
    run("fgmres_32", lambda: lat.solve_fgmres_dr(b, k=0, check=False, nkv=32, **kw))
    run("fgmres_dr_32_10", lambda: lat.solve_fgmres_dr(b, k=10, check=False, nkv=32, **kw))
    rec["speedup_dr_vs_fgcr_32"] = rec["fgcr_32"]["ms"] / rec["fgmres_dr_32_10"]["ms"]
    return rec


def summarise_pmc(fetch_csv, write_csv, out_json):
    """Turn two rocprofv3 --pmc runs of `bench.py --profile` (FETCH_SIZE, then WRITE_SIZE)
    into HBM bytes per launch per kernel.  The counters are scaled by what they read for the
    run's 1 GiB device copy (1 GiB read, 1 GiB written)."""
    import csv
    import hashlib

    def per_kernel(path, name):
        # the last 20 dispatches of each kernel: the final timing replay of its benchmark loop,
        # i.e. the launch variant whose duration bench.py reports
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == name]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        agg = {}
        for r in rows:
            agg.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
        return agg

    fetch_all, write_all = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    gib = float(1 << 30)
    # the 1 GiB copy is the largest copyBuffer dispatch of the run
    copy_f = max((v for k, vs in fetch_all.items() if "copyBuffer" in k for v in vs), default=gib)
    copy_w = max((v for k, vs in write_all.items() if "copyBuffer" in k for v in vs), default=gib)
    fetch = {k: v[-20:] for k, v in fetch_all.items()}
    write = {k: v[-20:] for k, v in write_all.items()}
    cf, cw = gib / copy_f, gib / copy_w
    src = os.path.join(ROOT, "paper_1109_4279_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(src)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(src, f), "rb").read())
    kernels = {}
    for k in fetch:
        if "wc::" not in k or k not in write:
            continue
        short = k.replace("void ", "").replace("wc::", "").split("(")[0]
        fb = cf * sum(fetch[k]) / len(fetch[k])
        wb = cw * sum(write[k]) / len(write[k])
        kernels[short] = {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
                          "launches": len(fetch[k])}
    rec = {"csrc_sha256": h.hexdigest(), "fetch_scale": cf, "write_scale": cw,
           "command": "rocprofv3 --pmc FETCH_SIZE|WRITE_SIZE --output-format csv -- python bench.py --profile "
                      "--steps 2 --warmup 1", "kernels": kernels}
    json.dump(rec, open(out_json, "w"), indent=1)
    return rec


# kernels of the profile report: (label, kernel, its figure in the bench record)
REPORT_LOOPS = [
    ("even/odd block solver `k_sap_eo<F32,1,cached>` (dominant kernel, 4 steps)", "k_sap_eo<1, 1, true>",
     lambda b: b["roofline"]["launch_ms"]),
    ("plain MR block solver `k_sap_mr<F32,1,cached,256>` (4 steps)", "k_sap_mr<1, 1, true, 256>",
     lambda b: b["roofline"]["plain_mr_half_sweep_ms"]),
    ("D_w FP64 `k_dirac<F64,1,staged>`", "k_dirac<0, 1, true>", lambda b: b["dirac"]["f64"]["ms"]),
    ("D_w FP32 `k_dirac<F32,1>`", "k_dirac<1, 1, false>", lambda b: b["dirac"]["f32"]["ms"]),
    ("D_w FP16 `k_dirac<F16,1>`", "k_dirac<2, 1, false>", lambda b: b["dirac"]["f16"]["ms"]),
    ("D_w BF16 `k_dirac<BF16,1>`", "k_dirac<3, 1, false>", lambda b: b["dirac"]["bf16"]["ms"]),
]
# kernels of the traffic table: (kernel, note, algorithmic read bytes per site)
REPORT_TRAFFIC = [
    ("k_sap_eo<1, 1, true>", "(one colour)", "864 per solved site = 432 per site"),
    ("k_sap_mr<1, 1, true, 256>", "(one colour)", "864 per solved site = 432 per site"),
    ("k_sap_eo<0, 1, false>", "(FP64, operator reloaded every phase)", "864 per site"),
    ("k_dirac<0, 1, true>", "(FP64, tile staged in LDS)", "1344"),
    ("k_dirac<1, 1, false>", "", "672"),
    ("k_dirac<2, 1, false>", "", "352"),
    ("k_dirac<3, 1, false>", "", "352"),
]


def _last_json_line(path):
    return json.loads([ln for ln in open(path).read().splitlines() if ln.startswith('{"metric"')][-1])


def profile_report(stats_dir, profiled_out, bench_out, fetch_csv, write_csv, traffic_json, out_md):
    """Markdown summary of one profiling pass of the 16^3 x 32 workload: the kernel
    statistics of `rocprofv3 --kernel-trace --stats -d STATS_DIR -o run -- bench.py --profile`
    (its stdout in PROFILED_OUT), the last-20-dispatch averages of the benchmark loops beside
    what bench.py printed (profiled and unprofiled: BENCH_OUT), and the HBM traffic record
    that `--summarise-pmc FETCH_CSV WRITE_CSV TRAFFIC_JSON` wrote."""
    import csv

    prof_cmd = "--profile --steps 2 --warmup 1"
    stats = list(csv.DictReader(open(os.path.join(stats_dir, "run_kernel_stats.csv"))))
    spans = {}
    for r in csv.DictReader(open(os.path.join(stats_dir, "run_kernel_trace.csv"))):
        spans.setdefault(r["Kernel_Name"], []).append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))

    def last20_us(kernel):
        for name, v in spans.items():
            if kernel in name:
                v = sorted(v)[-20:]
                return sum(e - s for s, e in v) / len(v) / 1e3
        return float("nan")

    pb, ub = _last_json_line(profiled_out), _last_json_line(bench_out)
    tk = json.load(open(traffic_json))
    V = 131072

    def pmc_cmd(counter, path):
        d, f = os.path.split(path)
        return (f"rocprofv3 --pmc {counter} --output-format csv -d {d} -o {f.split('_counter_collection')[0]} "
                f"-- python -u bench.py {prof_cmd}")

    out = ["# rocprofv3 summary: bench workload (16^3x32 mixed-precision SAP-FGCR), MI355X\n",
           "Kernel trace and statistics (durations in microseconds):\n",
           f"```\nrocprofv3 --kernel-trace --stats --output-format csv -d {stats_dir} -o run -- python -u bench.py "
           f"{prof_cmd}\n```",
           "The run holds 1 warm-up + 2 timed mixed solves with the even/odd block solver, the FP64\n"
           "solves with the even/odd and with the plain MR block solver, the mixed solve with the plain\n"
           "MR block solver, the D_w timing loops (2 warm-up + 2 x 20 graph-captured launches per\n"
           "precision) and the Schwarz half-sweep timing loops of both block solvers.  The solves'\n"
           "half-sweeps include the lighter first and last variants (no border update, no stores), so\n"
           "the all-dispatch average of a block solver is below its benchmark-loop figure.\n",
           "| kernel | calls | average | % of GPU time |\n|---|---|---|---|"]
    for r in stats[:14]:
        out.append(f"| `{r['Name']}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.1f} |")
    out += ["\nBenchmark-loop dispatches (last 20 of each kernel = the graph replay timed by `bench.py` with\n"
            "HIP events on the launch stream):\n",
            "| kernel | rocprofv3 avg (us) | bench.py (us) |\n|---|---|---|"]
    unprof = []
    for label, kernel, ms in REPORT_LOOPS:
        out.append(f"| {label} | {last20_us(kernel):.2f} | {ms(pb) * 1e3:.2f} |")
        unprof.append(f"{ms(ub) * 1e3:.2f}")
    out.append(f"\n(`bench.py` column: what the same profiled command printed; the unprofiled `python bench.py`\n"
               f"run printed {', '.join(unprof[:-1])} and {unprof[-1]} us.)\n\n"
               f"HBM traffic of the same dispatches from two counter runs (FETCH_SIZE, then WRITE_SIZE),\n"
               f"scaled by what the counters read for the run's 1 GiB device copy (fetch x {tk['fetch_scale']:.1f}, "
               f"write x {tk['write_scale']:.1f};\nthe exact factors are in `{os.path.basename(traffic_json)}`); "
               f"per launch and per lattice site (V = {V}):\n\n```\n{pmc_cmd('FETCH_SIZE', fetch_csv)}\n"
               f"{pmc_cmd('WRITE_SIZE', write_csv)}\npython bench.py --summarise-pmc {fetch_csv} {write_csv} "
               f"{traffic_json}\n```\n")
    out.append("| kernel | fetch B/site | write B/site | algorithmic read B/site |\n|---|---|---|---|")
    for kernel, note, alg in REPORT_TRAFFIC:
        v = tk["kernels"].get(kernel)
        if v is None:
            continue
        name = f"`{kernel}` {note}".rstrip()
        out.append(f"| {name} | {v['fetch_bytes'] / V:.0f} | {v['write_bytes'] / V:.0f} | {alg} |")
    # one timed mixed solve from the trace: solves open with the |b|^2 kernel; the first
    # warm-up-free one that runs the FP32 even/odd block solver, up to its first idle gap
    # above 2 ms
    trace = sorted((s0, e0, n.split("(")[0].replace("void ", "").replace("wc::", ""))
                   for n, v in spans.items() for s0, e0 in v)
    starts = [i for i, t in enumerate(trace) if t[2] == "k_norm2"]
    solves = []
    for j, i0 in enumerate(starts):
        seg = trace[i0:starts[j + 1] if j + 1 < len(starts) else len(trace)]
        for q in range(1, len(seg)):
            if seg[q][0] - seg[q - 1][1] > 2_000_000:
                seg = seg[:q]
                break
        if any(t[2] == "k_sap_eo<1, 1, true>" for t in seg):
            solves.append(seg)
    if len(solves) >= 2:
        seg = solves[1]
        span = (seg[-1][1] - seg[0][0]) / 1e6
        busy = sum(e0 - s0 for s0, e0, _ in seg) / 1e6
        per = {}
        for s0, e0, n in seg:
            per[n] = per.get(n, 0.0) + (e0 - s0) / 1e6
        out.append(f"\nOne timed mixed solve (the second with the FP32 even/odd block solver in the trace): "
                   f"{len(seg)} kernels,\n{busy:.2f} ms of kernels in a {span:.2f} ms span (idle between kernels "
                   f"{span - busy:.2f} ms, {100 * (span - busy) / span:.1f} %):\n")
        out.append("| kernel | ms | % of kernel time |\n|---|---|---|")
        for n, v in sorted(per.items(), key=lambda x: -x[1])[:8]:
            out.append(f"| `{n}` | {v:.3f} | {100 * v / busy:.1f} |")
    out.append(f"\nThis summary: `python bench.py --profile-report {stats_dir} {profiled_out} {bench_out} {fetch_csv} "
               f"{write_csv} {traffic_json} {out_md}`, where `{profiled_out}` holds the stdout of the kernel-trace "
               f"run and `{bench_out}` that of `python bench.py`.")
    open(out_md, "w").write("\n".join(out) + "\n")


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarise-pmc":
        summarise_pmc(sys.argv[2], sys.argv[3], sys.argv[4])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--profile-report":
        if len(sys.argv) != 9:
            sys.exit("usage: bench.py --profile-report STATS_DIR PROFILED_OUT BENCH_OUT FETCH_CSV WRITE_CSV "
                     "TRAFFIC_JSON OUT_MD")
        profile_report(*sys.argv[2:9])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--profile", action="store_true", help="short run for profilers: no CPU leg, few kernels")
    ap.add_argument("--no-extras", action="store_true", help="skip the 24^3x48 batch and 32^3x64 workloads")
    ap.add_argument("--profile-batch", action="store_true",
                    help="for profilers: only the batched 12-rhs 24^3x48 solve (one warm-up, one timed)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (sharding the lattice "
              "into sub-lattices with one halo exchange per Schwarz half-sweep is not implemented); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1109_4279_amd as wc
    import synth

    dev = torch.device("cuda:0")
    if args.profile_batch:
        dims = (48, 24, 24, 24)
        lat = wc.Lattice(torch.from_numpy(synth.gauge_field(dims)).to(dev), block=BLOCK, m0=M0, csw=CSW)
        pts = torch.from_numpy(synth.point_sources(dims)).to(dev)
        _, st, t = timed_solve(lat, pts, params(wc, "f16", True), torch)
        print(json.dumps({"workload": "batched 12 point sources, 24^3x48, FP16-storage even/odd SAP, FP64 FGCR",
                          "ms": t, "iters": max(x["iters"] for x in st),
                          "max_true_rel_residual": max(x["rel_true_res"] for x in st)}), flush=True)
        return
    if args.profile:
        # known-size copy (1 GiB read + 1 GiB written) that calibrates the FETCH_SIZE /
        # WRITE_SIZE counters of a profiled run
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    U_np = synth.gauge_field(DIMS)
    b_np = synth.gaussian_spinor(DIMS)
    U = torch.from_numpy(U_np).to(dev)
    b = torch.from_numpy(b_np).to(dev)
    lat = wc.Lattice(U, block=BLOCK, m0=M0, csw=CSW)
    V = lat.volume
    mixed = params(wc, "f32", True)

    for _ in range(args.warmup):
        lat.solve(b, mixed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(args.steps):
        x, st = lat.solve(b, mixed)
        stats.append(st[0])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    st = stats[-1]
    # the answer, checked with the library's own FP64 operator
    r = b - lat.apply_D(x)
    rel_res = (torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b)).item()
    flops = solve_flops(V, st["iters"], st["restarts"], NKV, NCY, NMR, eo=True)
    value = flops / (ms_per_step * 1e-3) / 1e9

    # FP64 on the same system with the same block solver and with MR on D_Lambda, and the
    # mixed solve with MR on D_Lambda
    x64, st64, tts_fp64 = timed_solve(lat, b, params(wc, "f64", True), torch)
    _, st64mr, tts_fp64_mr = timed_solve(lat, b, params(wc, "f64", False), torch)
    _, stmr, tts_mixed_mr = timed_solve(lat, b, params(wc, "f32", False), torch)
    rel_err = (torch.linalg.vector_norm(x - x64) / torch.linalg.vector_norm(x64)).item()

    # D_w per storage precision (HIP events inside the library, same stream)
    dw = {}
    for prec in ("f64", "f32", "f16", "bf16"):
        ms = lat.bench_dirac(prec=prec, nrhs=1, iters=20 if args.profile else 100)
        gbs = DW_BYTES[prec] * V / (ms * 1e-3) / 1e9
        dw[prec] = {"ms": ms, "GB/s": gbs, "Gflop/s": DW_FLOPS * V / (ms * 1e-3) / 1e9,
                    "frac_hbm": gbs / HBM_PEAK_GBS}
    # dominant kernel of the step: the FP32 Schwarz half-sweep (one colour, 4 steps of the
    # even/odd block solver); the unpreconditioned block solver's half-sweep beside it
    # the same half-sweep with no MR step: loads, border update, source and odd half, stores
    # (timed first, so that the last dispatches of the kernel in a profile are the nmr-step ones)
    ms_sap0 = lat.bench_sap(prec="f32", nrhs=1, nmr=0, eo=True, iters=20 if args.profile else 100)
    ms_sap = lat.bench_sap(prec="f32", nrhs=1, nmr=NMR, eo=True, iters=20 if args.profile else 100)
    ms_sap_mr = lat.bench_sap(prec="f32", nrhs=1, nmr=NMR, eo=False, iters=20 if args.profile else 100)
    sites = V // 2
    sap_bytes = SAP_BYTES_F32 * sites
    sap_flops = (half_sweep_flops_per_site(NMR, True) + BORDER_FLOPS_4444) * sites
    tf = sap_flops / (ms_sap * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": tf, "peak": FP32_SCALAR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tf / FP32_SCALAR_PEAK_TFLOPS, "traffic": measured_traffic("k_sap_eo<1, 1, true>"),
                "kernel": "k_sap_eo<F32, 1 rhs, cached> (one colour of 16^3x32, 4 steps)",
                "launch_ms": ms_sap, "alg_flops_per_launch": sap_flops, "alg_bytes_per_launch": sap_bytes,
                "hbm_GBps_alg": sap_bytes / (ms_sap * 1e-3) / 1e9,
                "frac_of_packed_fp32_peak": tf / FP32_PEAK_TFLOPS,
                "plain_mr_half_sweep_ms": ms_sap_mr}
    # two phases of the launch: every HBM byte moves in the set-up and the stores (nmr = 0
    # time); the MR steps run from registers and LDS (time per step from the difference)
    step_ms = (ms_sap - ms_sap0) / NMR
    step_flops = (DW_FLOPS + MR_VEC_FLOPS / 2) * sites
    setup_bytes = roofline["traffic"] if roofline["traffic"] else sap_bytes
    roofline["phases"] = {
        "setup_ms": ms_sap0, "step_ms": step_ms,
        "setup_GBps": setup_bytes / (ms_sap0 * 1e-3) / 1e9,
        "setup_bytes": "measured traffic" if roofline["traffic"] else "algorithmic",
        "step_TFLOPs": step_flops / (step_ms * 1e-3) / 1e12,
        "step_frac": step_flops / (step_ms * 1e-3) / 1e12 / FP32_SCALAR_PEAK_TFLOPS}

    extras = {}
    if not args.profile and not args.no_extras:
        extras = extra_workloads(wc, torch, dev)

    cpu = None
    if not args.no_cpu and not args.profile:
        cpu = cpu_baseline(U_np, b_np)

    out = {
        "metric": "D_w GB/s & Gflop/s vs HBM roofline; FGCR time-to-1e-10 (mixed vs FP64)",
        "value": value,
        "unit": "Gflop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "SAP-FGCR solve to 1e-10, 16^3x32, eps=0.3 gauge, m0=-0.1, c_sw=1, "
                               "blocks 4^4, nmr=4 (even/odd block solver), ncy=5, nkv=16, 1 Gaussian rhs, "
                               "FP32 SAP / FP64 outer",
                   "lattice": list(DIMS), "block": list(BLOCK), "parallelism": "single GPU"},
        "tts_mixed_ms": ms_per_step,
        "tts_fp64_ms": tts_fp64,
        "speedup_mixed_vs_fp64": tts_fp64 / ms_per_step,
        "tts_fp64_mr_ms": tts_fp64_mr,
        "speedup_mixed_vs_fp64_mr": tts_fp64_mr / ms_per_step,
        "tts_mixed_mr_ms": tts_mixed_mr,
        "iters_mixed": st["iters"], "restarts_mixed": st["restarts"],
        "iters_fp64": st64[0]["iters"], "iters_fp64_mr": st64mr[0]["iters"], "iters_mixed_mr": stmr[0]["iters"],
        "true_rel_residual": rel_res, "rel_err_mixed_vs_fp64": rel_err,
        "dirac": dw,
        "roofline": roofline,
        "cpu_baseline": cpu,
        **extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
