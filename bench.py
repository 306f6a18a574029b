"""Benchmark of the Wilson-clover SAP-FGCR hot path on one MI355X.

One step = the batched mixed-precision solve of the 12 spin-colour point sources on the
24^3 x 48 lattice (gauge recipe eps = 0.3, m0 = -0.1, c_sw = 1) to a true FP64 residual of
1e-10 per right-hand side: FP32 arithmetic in the Schwarz preconditioner (even/odd block
solver, 4 steps, 5 cycles) on 16-bit or FP32 storage, FP64 FGCR (restart 16), every kernel
one launch over all 12 right-hand sides and each restart cycle one captured hipGraph.
Storage precision, Schwarz block shape and right-hand-side tiles are chosen by timing
before the timed steps (the block shape and tiles by the library's autotuners); inputs are
resident on the device.

`value` is right-hand sides solved per second (12 / step time).  Beside it:
  * the speedup per right-hand side against 12 single-rhs solves with the plain FP64
    method on the same lattice (and against FP64 with the same block solver);
  * the roofline record of the step's dominant kernel (the block solver's half-sweep over
    all 12 right-hand sides), executed flops and algorithmic bytes per launch, bound by
    arithmetic intensity against the ridge of the FP32 vector peak and 8 TB/s;
  * D_w GB/s and Gflop/s per storage precision on 16^3 x 32, 24^3 x 48 and 32^3 x 64, and
    with the 12 right-hand sides of 24^3 x 48 in one launch;
  * the uneven batch {8^3 x 16, 12^3 x 24, 16^3 x 32} x 4 Gaussian rhs as one solve;
  * the 32^3 x 64 solves on every storage with their error against an independent FP64
    reference solve, the 16^3 x 32 solves, the force of S = phi^dag (D^dag D)^-1 phi on
    16^3 x 32, and FGCR against FGMRES-DR close to the critical mass;
  * the FP64 oracle on the host's cores for a bounded sample of the step's workload.
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

M0, CSW = -0.1, 1.0
NKV, NCY, NMR, TOL = 16, 5, 4, 1e-10
C4_DIMS = (48, 24, 24, 24)
C2_DIMS = (32, 16, 16, 16)
C3_DIMS = (64, 32, 32, 32)
UNEVEN = [(16, 8, 8, 8), (24, 12, 12, 12), (32, 16, 16, 16)]
BLOCK = (4, 4, 4, 4)
HBM_PEAK_GBS = 8000.0
FP32_PACKED_PEAK_TFLOPS = 157.3
# FP32 rate of the kernels as built (packed FP32 instructions switched off): 256 CUs x 4
# SIMDs x 16 lanes x 2 flop per FMA x 2.4 GHz
FP32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
RIDGE_FLOP_PER_B = FP32_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)

DW_FLOPS = 1320 + 504          # nominal flops per site of D_w
HOP_FLOPS = 144                # project 12 + SU(3) x half spinor 132 per hop
ACC_FLOPS = 24                 # one spinor accumulate
CLOVER_FLOPS = 504             # both 6x6 chiral blocks
MR_VEC_FLOPS = 336             # per site and MR step: <q,rho>, <q,q>, z += a rho, rho -= a q
# bytes per site of one storage precision: spinor, links (4), clover (2 blocks), scales included
SPINOR_B = {"f64": 192, "f32": 96, "f16": 52, "bf16": 52}
LINKS_B = {"f64": 576, "f32": 288, "f16": 148, "bf16": 148}
CLOVER_B = {"f64": 576, "f32": 288, "f16": 152, "bf16": 152}


def dw_bytes(prec, tile=1):
    """Algorithmic bytes per site and rhs of D_w: spinor in and out, plus links and clover
    once per tile of `tile` right-hand sides."""
    return 2 * SPINOR_B[prec] + (LINKS_B[prec] + CLOVER_B[prec]) / tile


def mean_inblock_hops(block):
    return sum(2.0 * (b - 1) / b for b in block)


def dlambda_flops(block):
    """Executed flops per site of the Dirichlet block operator (hops to other blocks dropped)."""
    h = mean_inblock_hops(block)
    return HOP_FLOPS * h + ACC_FLOPS * (h - 1) + CLOVER_FLOPS


def half_sweep_flops(block, nmr, eo, executed=True):
    """Flops per solved site of one Schwarz half-sweep.  Executed: the block operator as
    applied (in-block hops only), the border update's hops out of the block, psi += z.
    Even/odd block solver: an application of the Schur complement touches every block site
    once (hops and a 6x6 clover pair) and the MR vector work runs on the even half; the
    source and the odd half of the solution add one block sweep.  Nominal: D_Lambda counted
    as the full 1824 flops of D_w."""
    op = dlambda_flops(block) if executed else DW_FLOPS
    border = (8 - mean_inblock_hops(block)) * (HOP_FLOPS + ACC_FLOPS)
    if eo:
        return nmr * (op + MR_VEC_FLOPS / 2) + op + 12 + border + 24
    return nmr * (op + MR_VEC_FLOPS) + border + 24


def half_sweep_bytes(prec, tile=1):
    """Algorithmic bytes per solved site and rhs of one half-sweep: the block operator (links
    and clover) once per tile of rhs; residual in and out, solution out, psi in and out, the
    neighbouring blocks' solution read once."""
    return (LINKS_B[prec] + CLOVER_B[prec]) / tile + 6 * SPINOR_B[prec]


def solve_flops(V, iters, restarts, nkv, ncy, nmr, block, eo, executed=True):
    """Flops of a restarted SAP-FGCR solve of one rhs with `iters` iterations over `restarts`
    cycles (Gram-Schmidt counted as one classical pass)."""
    dflops = DW_FLOPS
    f = 0.0
    left = iters
    for _ in range(max(restarts, 1)):
        kd = min(nkv, left)
        left -= kd
        for k in range(kd):
            # one SAP application: 2 ncy half-sweeps, each over half of the sites; scaling in/out
            f += ncy * half_sweep_flops(block, nmr, eo, executed) + 48
            f += dflops
            f += 2 * 96 * k + 144 + 168
        f += 96 * kd + dflops + 72
    return f * V


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


SAMPLE_DIMS = (8, 24, 24, 24)  # a 24^3 x 8 slab: 1/6 of 24^3 x 48 with the same 4^4 blocks
SAMPLE_SCALE = 6


def _oracle_sample(args):
    """A bounded sample of one rhs of the step's workload in the FP64 oracle, single-threaded:
    one D_w and one Schwarz half-sweep of the even/odd block solver on a 24^3 x 8 slab of
    the lattice (the block solves are independent, so the half-sweep's cost is linear in the
    number of blocks).  Returns their wall times (the clover set-up is not timed)."""
    dims, seed = args
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import dirac, solvers
    with threadpool_limits(limits=1):
        U = synth.gauge_field(dims)
        A = dirac.clover_matrix(U, M0, CSW)
        Ainv = dirac.clover_inverse(A)
        b = synth.gaussian_spinor(dims, seed=seed)
        t0 = time.perf_counter()
        dirac.apply_D(U, A, b)
        t_d = time.perf_counter() - t0
        t0 = time.perf_counter()
        solvers.mr_blocks_eo(U, A, b, BLOCK, 0, NMR, 1, Ainv)
        t_hs = time.perf_counter() - t0
    return t_d, t_hs


def cpu_baseline(iters, restarts, workers):
    """The FP64 oracle on the host, in the headline's unit: its time for one of the step's
    right-hand sides is estimated from a bounded sample (one D_w and one even/odd Schwarz
    half-sweep on 24^3 x 48, measured single-threaded), as iters x (2 ncy half-sweeps + one
    D) + one D per restart; Gram-Schmidt is left out, which favours the oracle.  The
    all-core leg runs the sample in one process per core (independent right-hand sides)."""
    import concurrent.futures as cf
    import multiprocessing as mp

    def per_rhs(t_d, t_hs):
        return SAMPLE_SCALE * (iters * (2 * NCY * t_hs + t_d) + restarts * t_d)

    vs = SAMPLE_DIMS[0] * SAMPLE_DIMS[1] * SAMPLE_DIMS[2] * SAMPLE_DIMS[3]
    t0 = time.perf_counter()
    t_d, t_hs = _oracle_sample((SAMPLE_DIMS, 5678))
    t_one = time.perf_counter() - t0
    one = 1.0 / per_rhs(t_d, t_hs)
    rec = {"value": one, "unit": "rhs/s", "cores": 1, "kind": "oracle",
           "sample": f"numpy FP64 oracle, 1 thread, on a 24^3x8 slab (1/{SAMPLE_SCALE} of 24^3x48, same 4^4 "
                     f"blocks): one D_w ({t_d:.2f} s) and one even/odd Schwarz half-sweep with {NMR} steps "
                     f"({t_hs:.2f} s); one rhs of the step = {SAMPLE_SCALE} x [{iters} x ({2 * NCY} half-sweeps + D) "
                     f"+ {restarts} D] = {per_rhs(t_d, t_hs):.0f} s (Gram-Schmidt not counted)",
           "cpu_model": cpu_model(), "host_cores": host_cores(), "oracle_dirac_s_per_site": t_d / vs,
           "oracle_dirac_GBps": dw_bytes("f64") * vs / t_d / 1e9,
           "oracle_dirac_Gflops": DW_FLOPS * vs / t_d / 1e9, "sample_wall_s": t_one}
    if workers > 1:
        t0 = time.perf_counter()
        with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
            res = list(ex.map(_oracle_sample, [(SAMPLE_DIMS, 5678 + i) for i in range(workers)]))
        wall = time.perf_counter() - t0
        slowest = max(per_rhs(a, b) for a, b in res)
        rec["all_cores"] = {"value": workers / slowest, "unit": "rhs/s", "cores": workers,
                            "per_rhs_s": slowest, "wall_s": wall,
                            "note": "one process per core, each the single-thread sample on its own rhs; "
                                    "aggregate = processes / slowest per-rhs estimate"}
    return rec


def csrc_sha256():
    """Digest of the kernel sources (every .hip and .h under csrc/), stored with each counter
    record so that a record taken on other kernels is not used."""
    import hashlib
    src = os.path.join(ROOT, "paper_1109_4279_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(src)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(src, f), "rb").read())
    return h.hexdigest()


def _current_record(path, kernel):
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", path)))
    except (OSError, ValueError):
        return None
    if rec.get("csrc_sha256") != csrc_sha256() or kernel not in rec.get("kernels", {}):
        return None
    return rec["kernels"][kernel]


def measured_traffic(kernel, path):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    record at `path`, or None when the kernel sources changed since it was taken."""
    r = _current_record(path, kernel)
    return None if r is None else r["bytes_per_launch"]


def measured_valu(kernel, path):
    """VALU occupancy of `kernel` from the committed SQ counter record at `path` (see
    valu_record), or None when the kernel sources changed since it was taken."""
    return _current_record(path, kernel)


def valu_record(csv_path, out_json, kernel="k_sap_eo<3, 1, false>", simds=1024, xcds=8):
    """VALU occupancy of the block solver from a rocprofv3 --pmc SQ_INSTS_VALU GRBM_GUI_ACTIVE
    run of `bench.py --profile`, whose last timing loops are 20+ launches without MR steps
    and then 20+ with them: SQ_INSTS_VALU x 4 cycles per wave64 instruction over the SIMDs
    and the launch's cycles per XCD (GRBM_GUI_ACTIVE / xcds), for the launch with MR steps,
    the one without (set-up, odd half, stores) and their difference (the MR steps)."""
    import csv
    per = {}
    for r in csv.DictReader(open(csv_path)):
        short = r["Kernel_Name"].replace("void ", "").replace("wc::", "").split("(")[0]
        if short == kernel:
            per.setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
    ids = sorted(per)
    last = per[ids[-1]]["SQ_INSTS_VALU"]
    with_mr = ids[-20:]
    without = [i for i in ids if abs(per[i]["SQ_INSTS_VALU"] - last) > 0.01 * last][-20:]

    def mean(sel, c):
        return sum(per[i][c] for i in sel) / len(sel)

    def busy(v, g):
        return v * 4 / (simds * g / xcds)

    v4, g4 = mean(with_mr, "SQ_INSTS_VALU"), mean(with_mr, "GRBM_GUI_ACTIVE")
    v0, g0 = mean(without, "SQ_INSTS_VALU"), mean(without, "GRBM_GUI_ACTIVE")
    rec = {"csrc_sha256": csrc_sha256(),
           "command": "rocprofv3 --pmc SQ_INSTS_VALU ... GRBM_GUI_ACTIVE --output-format csv -- python bench.py --profile",
           "kernels": {kernel: {"valu_busy_launch": busy(v4, g4), "valu_busy_without_mr_steps": busy(v0, g0),
                                "valu_busy_mr_steps": busy(v4 - v0, g4 - g0), "valu_instructions_per_launch": v4}}}
    json.dump(rec, open(out_json, "w"), indent=1)
    return rec


def sync_time(torch, f):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = f()
    torch.cuda.synchronize()
    return out, (time.perf_counter() - t0) * 1e3


def params(wc, sap_prec, eo, **kw):
    base = dict(nkv=NKV, ncy=NCY, nmr=NMR, tol=TOL, sap_prec=sap_prec, eo=int(eo), use_graph=1)
    base.update(kw)
    return wc.default_params(**base)


def timed_solve(lat, b, p, torch):
    lat.solve(b, p)
    (x, st), ms = sync_time(torch, lambda: lat.solve(b, p))
    return x, st, ms


def single_solves(lat, srcs, p, torch):
    """Mean time per rhs of solving the sources one at a time (after a warm-up solve)."""
    lat.solve(srcs[0].contiguous(), p)
    t, iters = 0.0, []
    for r in range(srcs.shape[0]):
        src = srcs[r].contiguous()
        (_, st1), ms = sync_time(torch, lambda: lat.solve(src, p))
        t += ms / srcs.shape[0]
        iters.append(st1[0]["iters"])
    return t, max(iters)


COPY_GBS = {}  # measured device-copy rate, the second denominator of the D_w fractions


def copy_bandwidth(torch, dev, gib=1, reps=10):
    """Read + write rate of a plain device copy of `gib` GiB: torch's copy kernel, `reps`
    copies back to back between two events on torch's stream (the one the copies run on),
    after one warm-up; in GB/s."""
    n = gib * (1 << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * gib * (1 << 30) / (ms * 1e-3) / 1e9


def dirac_rates(lat, V, precs, nrhs=1, iters=50):
    out = {}
    copy = COPY_GBS.get("GB/s")
    for prec in precs:
        ms = lat.bench_dirac(prec=prec, nrhs=nrhs, iters=iters)
        rec = {"ms": ms, "Gflop/s": DW_FLOPS * V * nrhs / (ms * 1e-3) / 1e9}
        if nrhs == 1:
            gbs = dw_bytes(prec) * V / (ms * 1e-3) / 1e9
            rec.update({"GB/s": gbs, "frac_hbm": gbs / HBM_PEAK_GBS})
            if copy:
                rec["frac_copy"] = gbs / copy
        else:
            # the operator counted once per rhs tile of the kernel, and once for all nrhs
            tile = lat_tile(lat, prec)
            g_tile = dw_bytes(prec, tile) * V * nrhs / (ms * 1e-3) / 1e9
            g_all = dw_bytes(prec, nrhs) * V * nrhs / (ms * 1e-3) / 1e9
            rec.update({"rhs_per_lane": tile, "GB/s": g_tile, "frac_hbm": g_tile / HBM_PEAK_GBS,
                        f"GB/s_operator_once_per_{nrhs}_rhs": g_all,
                        f"frac_hbm_operator_once_per_{nrhs}_rhs": g_all / HBM_PEAK_GBS})
        out[prec] = rec
    return out


_TILES = {}


def lat_tile(lat, prec):
    return _TILES.get((id(lat), prec), 1)


def tune_c4(wc, torch, lat, pts):
    """Tuning before the timed steps (not timed): the Schwarz block shape (library autotuner,
    one short single-rhs solve per valid shape), the rhs tiles (library autotuner, per
    storage), the storage precision of the preconditioner (one batched solve each), then the
    storage of the FGCR Krylov basis: FP64, or F32 with cycles that end at a 1e-6 drop of
    the residual (the single-precision recursion between FP64 restarts; one solve each)."""
    t0 = time.perf_counter()
    block = lat.autotune_block(params(wc, "f32", True))
    tiles, times = {}, {}
    for sp in ("f32", "f16", "bf16"):
        tiles[sp] = lat.autotune(12, prec=sp)
        _, _, times[sp] = timed_solve(lat, pts, params(wc, sp, True), torch)
    best = min(times, key=times.get)
    tiles[best] = lat.autotune(12, prec=best)  # the chosen storage's tiles stay in the context
    _TILES[(id(lat), best)] = tiles[best][0]
    _TILES[(id(lat), "f64")] = tiles[best][1]
    basis_ms = {}
    for qp in ("f64", "f32"):
        _, _, basis_ms[qp] = timed_solve(lat, pts, params(wc, best, True, basis_prec=qp), torch)
    basis = min(basis_ms, key=basis_ms.get)
    return {"block": list(block), "storage": best, "tiles": tiles, "trial_ms": times, "basis": basis,
            "basis_trial_ms": basis_ms, "tuning_s": time.perf_counter() - t0}


def roofline_record(lat, V, prec, nrhs, block, label, tile=1):
    """Roofline of the block solver's half-sweep (one colour, NMR steps, even/odd) timed
    inside the library with HIP events on its launch stream; the block operator counts once
    per tile of `tile` right-hand sides (the rhs a work-group shares it across)."""
    ms0 = lat.bench_sap(prec=prec, nrhs=nrhs, nmr=0, eo=True, iters=20)
    ms = lat.bench_sap(prec=prec, nrhs=nrhs, nmr=NMR, eo=True, iters=20)
    sites = V // 2 * nrhs
    flops = half_sweep_flops(block, NMR, True) * sites
    nominal = half_sweep_flops(block, NMR, True, executed=False) * sites
    byts = half_sweep_bytes(prec, tile) * sites
    tf = flops / (ms * 1e-3) / 1e12
    ai = flops / byts
    bound = "alu" if ai > RIDGE_FLOP_PER_B else "hbm"
    rec = {"bound": bound, "kernel": label, "launch_ms": ms,
           "alg_flops_per_launch": flops, "alg_bytes_per_launch": byts,
           "nominal_flops_per_launch": nominal, "arith_intensity": ai, "ridge": RIDGE_FLOP_PER_B,
           "TFLOPs_executed": tf, "frac_of_fp32_peak": tf / FP32_PEAK_TFLOPS,
           "frac_of_packed_fp32_peak": tf / FP32_PACKED_PEAK_TFLOPS,
           "GBps_alg": byts / (ms * 1e-3) / 1e9, "frac_hbm": byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    if bound == "alu":
        rec.update({"achieved": tf, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tf / FP32_PEAK_TFLOPS})
    else:
        g = rec["GBps_alg"]
        rec.update({"achieved": g, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": g / HBM_PEAK_GBS})
    step_ms = (ms - ms0) / NMR
    step_flops = (dlambda_flops(block) + MR_VEC_FLOPS / 2) * sites
    rec["phases"] = {"setup_and_stores_ms": ms0, "mr_step_ms": step_ms,
                     "mr_step_TFLOPs": step_flops / (step_ms * 1e-3) / 1e12}
    return rec


def extra_workloads(wc, torch, dev, storage, lat_c4, pts):
    import synth
    out = {}
    # the plain device copy's rate: the second denominator of the D_w fractions
    COPY_GBS["GB/s"] = copy_bandwidth(torch, dev)
    out["device_copy_GBps"] = COPY_GBS["GB/s"]
    # D_w on every size, one rhs; and the 12 rhs of 24^3 x 48 in one launch
    out["dirac_24c48"] = dirac_rates(lat_c4, 663552, ("f64", "f32", "f16", "bf16"))
    out["dirac_24c48_12rhs"] = dirac_rates(lat_c4, 663552, ("f64", storage), nrhs=12, iters=10)
    # 16^3 x 32: the plain-FP64 configuration and the mixed solve on the same system
    lat = wc.Lattice(torch.from_numpy(synth.gauge_field(C2_DIMS)).to(dev), block=BLOCK, m0=M0, csw=CSW)
    b = torch.from_numpy(synth.gaussian_spinor(C2_DIMS)).to(dev)
    c2 = {"dirac": dirac_rates(lat, 131072, ("f64", "f32", "f16", "bf16"), iters=100)}
    for name, sp, eo, qp in (("fp64_mr", "f64", 0, "f64"), ("fp64_eo", "f64", 1, "f64"),
                             ("mixed_f32_eo", "f32", 1, "f64"), ("mixed_f32_eo_f32_basis", "f32", 1, "f32")):
        _, st, ms = timed_solve(lat, b, params(wc, sp, eo, basis_prec=qp), torch)
        c2[name] = {"ms": ms, "iters": st[0]["iters"], "restarts": st[0]["restarts"],
                    "true_rel_residual": st[0]["rel_true_res"]}
    c2["roofline_k_sap_eo_f32_cached"] = roofline_record(lat, 131072, "f32", 1, BLOCK,
                                                          "k_sap_eo<F32, 1 rhs, cached>, 16^3x32, one colour")
    # the force of S = phi^dag (D^dag D)^-1 phi (two solves + the force kernel)
    phi = torch.from_numpy(synth.gaussian_spinor(C2_DIMS, seed=synth.FORCE_PHI_SEED)).to(dev)
    for name, sp in (("force_mixed_f32", "f32"), ("force_fp64", "f64")):
        p = params(wc, sp, True)
        lat.force(phi, p)
        (_, _, _, st), ms = sync_time(torch, lambda: lat.force(phi, p))
        c2[name] = {"ms": ms, "solve_iters": [s["iters"] for s in st]}
    Y = torch.from_numpy(synth.gaussian_spinor(C2_DIMS, seed=1)).to(dev)
    lat.link_grad(Y, b)
    _, ms = sync_time(torch, lambda: [lat.link_grad(Y, b) for _ in range(10)])
    c2["link_derivative_ms"] = ms / 10
    out["workload_16c32"] = c2
    out["near_critical_16c32"] = near_critical(wc, torch, lat.block, dev)
    out["near_critical_quenched_16c32"] = near_critical_quenched(wc, torch, dev, lat.block)
    del lat, b, phi
    # the uneven batch, one batched solve (block shapes chosen by the block autotuner)
    lats, bs = [], []
    for i, d in enumerate(UNEVEN):
        la = wc.Lattice(torch.from_numpy(synth.gauge_field(d, seed=synth.GAUGE_SEED + i)).to(dev), block=BLOCK
                        if d != (24, 12, 12, 12) else (4, 3, 3, 3), m0=M0, csw=CSW)
        la.autotune_block(params(wc, storage, True))
        lats.append(la)
        bs.append(torch.from_numpy(synth.gaussian_spinor(d, nrhs=4, seed=synth.RHS_SEED + i)).to(dev))
    ub = {"lattices": [list(d) for d in UNEVEN], "blocks": [list(la.block) for la in lats], "rhs_per_lattice": 4,
          "storage": storage}
    for qp, tag in (("f64", ""), ("f32", "_f32_basis")):
        p = params(wc, storage, True, basis_prec=qp)
        wc.solve_batch(lats, bs, p)
        (_, st), ms = sync_time(torch, lambda: wc.solve_batch(lats, bs, p))
        single = 0.0
        for la, bb in zip(lats, bs):
            la.solve(bb, p)
            _, t1 = sync_time(torch, lambda: la.solve(bb, p))
            single += t1
        ub.update({"batched_ms" + tag: ms, "separate_solves_ms" + tag: single,
                   "max_iters" + tag: max(s["iters"] for s in st),
                   "max_true_rel_residual" + tag: max(s["rel_true_res"] for s in st)})
    out["uneven_batch"] = ub
    del lats, bs
    # 32^3 x 64: every storage, and the error against an independent FP64 reference (the
    # plain MR block solver to 1e-12: another iteration than the mixed solves')
    lat = wc.Lattice(torch.from_numpy(synth.gauge_field(C3_DIMS)).to(dev), block=BLOCK, m0=M0, csw=CSW)
    b = torch.from_numpy(synth.gaussian_spinor(C3_DIMS)).to(dev)
    rec = {"dirac": dirac_rates(lat, 2097152, ("f64", "f32", "f16", "bf16"), iters=20)}
    xref, stref = lat.solve(b, params(wc, "f64", False, tol=1e-12))
    rec["reference"] = {"method": "FP64 SAP-FGCR, MR on D_Lambda, tol 1e-12",
                        "true_rel_residual": stref[0]["rel_true_res"], "iters": stref[0]["iters"]}
    nref = torch.linalg.vector_norm(xref)
    _, st, ms = timed_solve(lat, b, params(wc, "f64", False), torch)
    rec["fp64_mr"] = {"ms": ms, "iters": st[0]["iters"]}
    for name, sp, qp in (("fp64_eo", "f64", "f64"), ("f32", "f32", "f64"), ("f16", "f16", "f64"),
                         ("bf16", "bf16", "f64"), ("bf16_f32_basis", "bf16", "f32")):
        x, st, ms = timed_solve(lat, b, params(wc, sp, True, basis_prec=qp), torch)
        rec[name] = {"ms": ms, "iters": st[0]["iters"], "true_rel_residual": st[0]["rel_true_res"],
                     "rel_err_vs_fp64_reference": (torch.linalg.vector_norm(x - xref) / nref).item()}
    out["solve_32c64"] = rec
    del lat, b, xref
    return out


def near_critical(wc, torch, block, dev):
    """The regime of the paper's Fig. 1: m0 = -0.178, close to the critical mass of the
    synthetic eps = 0.3 field on 16^3 x 32.  FGCR with restart 16 and 32 against FGMRES-DR
    with 32 vectors of which 10 are deflated; FP32 even/odd SAP, FP64 outer, tol 1e-10."""
    import synth
    m0 = -0.178
    lat = wc.Lattice(torch.from_numpy(synth.gauge_field(C2_DIMS)).to(dev), block=block, m0=m0, csw=CSW)
    b = torch.from_numpy(synth.gaussian_spinor(C2_DIMS)).to(dev)
    rec = {"m0": m0}

    def run(name, f):
        f()
        (_, st), ms = sync_time(torch, f)
        rec[name] = {"ms": ms, "iters": st[0]["iters"], "restarts": st[0]["restarts"],
                     "true_rel_residual": st[0]["rel_true_res"], "status": st[0]["status"],
                     "gram_schmidt_second_passes": st[0]["reorth"]}

    kw = dict(ncy=NCY, nmr=NMR, tol=TOL, sap_prec="f32", eo=1, maxit=3000)
    run("fgcr_16", lambda: lat.solve(b, check=False, nkv=16, **kw))
    run("fgcr_32", lambda: lat.solve(b, check=False, nkv=32, **kw))
    run("fgmres_32", lambda: lat.solve_fgmres_dr(b, k=0, check=False, nkv=32, **kw))
    run("fgmres_dr_32_10", lambda: lat.solve_fgmres_dr(b, k=10, check=False, nkv=32, **kw))
    rec["speedup_dr_vs_fgcr_32"] = rec["fgcr_32"]["ms"] / rec["fgmres_dr_32_10"]["ms"]
    return rec


QUENCHED_BETA = 6.0
QUENCHED_CSW = 1.769  # non-perturbative c_sw at beta = 6.0 (ALPHA, Nucl. Phys. B 491 (1997) 323)


def critical_mass(wc, torch, U, dims, csw, block, m0_ref, dev, nev=12, seed=None):
    """Estimate of the critical bare mass of one gauge field by shift-invert Arnoldi: nev
    steps of Arnoldi (modified Gram-Schmidt, FP64 on the device) on D(m0_ref)^-1, each
    application a solve of the library's FGMRES-DR (FP32 even/odd SAP, 1e-10); the Ritz
    values theta of the small Hessenberg matrix give eigenvalue estimates 1/theta of
    D(m0_ref) closest to zero (conjugate pairs resolved, as D is gamma_5-hermitian).  The
    spectrum moves rigidly with m0, so the estimate closest to zero, lambda, reaches the
    imaginary axis at m0_c = m0_ref - Re lambda (the critical mass when it is real).
    Returns (m0_c, estimates sorted by modulus as [re, im] pairs)."""
    import numpy as np

    import synth
    lat = wc.Lattice(U, block=block, m0=m0_ref, csw=csw)
    v = torch.from_numpy(synth.gaussian_spinor(dims, seed=synth.RHS_SEED if seed is None else seed)).to(dev)
    V = [v / torch.linalg.vector_norm(v)]
    H = np.zeros((nev + 1, nev), dtype=np.complex128)
    for j in range(nev):
        w, _st = lat.solve_fgmres_dr(V[j], k=10, nkv=32, tol=1e-10, sap_prec="f32", eo=1, ncy=NCY, nmr=NMR,
                                     maxit=4000)
        for i in range(j + 1):
            h = torch.vdot(V[i].flatten(), w.flatten())
            H[i, j] = complex(h)
            w = w - h * V[i]
        H[j + 1, j] = float(torch.linalg.vector_norm(w))
        V.append(w / H[j + 1, j])
    del lat, V
    lam = 1.0 / np.linalg.eigvals(H[:nev, :nev])
    lam = lam[np.argsort(np.abs(lam))]
    return m0_ref - lam[0].real, [[z.real, z.imag] for z in lam]


def near_critical_quenched(wc, torch, dev, block):
    """The near-critical stress workload on a self-generated ensemble: a quenched 16^3 x 32
    field at beta = 6.0 (Wilson action; cold start, 20 x (1 heatbath + 4 overrelaxation)
    sweeps on the GPU), c_sw = 1.769, its critical mass estimated by shift-invert Arnoldi (two
    stages, the second 0.02 above the first estimate), then FGCR(16), FGCR(32) and
    FGMRES-DR(32, 10) on a Gaussian source at 0.02, 0.005 and 0.001 above it (FP32 even/odd
    SAP, FP64 outer, tol 1e-10, maxit 3000): the regime of Fig. 1, where restarted GCR slows
    down and deflated restarts keep the low modes.  FGCR(32) also runs with the
    single-precision recursion (F32 basis) to show what it does near the critical mass."""
    import synth
    from synth import quenched
    t0 = time.perf_counter()
    hist = []
    U = quenched.ensemble(C2_DIMS, beta=QUENCHED_BETA, ntherm=20, nor=4, device=dev, history=hist)
    torch.cuda.synchronize()
    rec = {"ensemble": {"dims": list(C2_DIMS), "beta": QUENCHED_BETA, "csw": QUENCHED_CSW,
                        "sweeps": "20 x (1 heatbath + 4 overrelaxation), cold start",
                        "generation_s": time.perf_counter() - t0, "plaquette_history": hist}}
    c1, l1 = critical_mass(wc, torch, U, C2_DIMS, QUENCHED_CSW, block, -0.25, dev)
    c2, l2 = critical_mass(wc, torch, U, C2_DIMS, QUENCHED_CSW, block, c1 + 0.02, dev)
    rec["critical_mass"] = {"method": "shift-invert Arnoldi, 12 solves per stage",
                            "stage1": {"m0_ref": -0.25, "m0_c": c1, "lowest_eigenvalues": l1[:6]},
                            "stage2": {"m0_ref": c1 + 0.02, "m0_c": c2, "lowest_eigenvalues": l2[:6]},
                            "estimate": c2}
    b = torch.from_numpy(synth.gaussian_spinor(C2_DIMS)).to(dev)
    kw = dict(ncy=NCY, nmr=NMR, tol=TOL, sap_prec="f32", eo=1, maxit=3000)
    lam2 = [complex(a, bb) for a, bb in l2]
    for dm in (0.02, 0.005, 0.001):
        lat = wc.Lattice(U, block=block, m0=c2 + dm, csw=QUENCHED_CSW)
        # the estimated smallest |eigenvalue| of D at this mass (the spectrum shifted by m0)
        r = {"m0": c2 + dm, "smallest_abs_eigenvalue": min(abs(z + (c2 + dm) - (c1 + 0.02)) for z in lam2)}

        def run(name, f):
            f()
            (_, st), ms = sync_time(torch, f)
            r[name] = {"ms": ms, "iters": st[0]["iters"], "restarts": st[0]["restarts"],
                       "true_rel_residual": st[0]["rel_true_res"], "status": st[0]["status"],
                       "gram_schmidt_second_passes": st[0]["reorth"]}

        run("fgcr_16", lambda: lat.solve(b, check=False, nkv=16, **kw))
        run("fgcr_32", lambda: lat.solve(b, check=False, nkv=32, **kw))
        run("fgcr_32_f32_basis", lambda: lat.solve(b, check=False, nkv=32, basis_prec="f32", **kw))
        run("fgmres_dr_32_10", lambda: lat.solve_fgmres_dr(b, k=10, check=False, nkv=32, **kw))
        r["speedup_dr_vs_fgcr_32"] = r["fgcr_32"]["ms"] / r["fgmres_dr_32_10"]["ms"]
        rec[f"dm_{dm}"] = r
        del lat
    del U
    return rec


def summarise_pmc(fetch_csv, write_csv, out_json, kernels_of_interest=None):
    """Turn two rocprofv3 --pmc runs of `bench.py --profile` (FETCH_SIZE, then WRITE_SIZE)
    into HBM bytes per launch per kernel.  The counters are scaled by what they read for the
    run's 1 GiB device copy (1 GiB read, 1 GiB written); each kernel's figure is the mean of
    its last 20 dispatches (the timing loop whose duration bench.py reports)."""
    import csv

    def per_kernel(path, name):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == name]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        agg = {}
        for r in rows:
            agg.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
        return agg

    fetch_all, write_all = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    gib = float(1 << 30)
    copy_f = max((v for k, vs in fetch_all.items() if "copyBuffer" in k for v in vs), default=gib)
    copy_w = max((v for k, vs in write_all.items() if "copyBuffer" in k for v in vs), default=gib)
    fetch = {k: v[-20:] for k, v in fetch_all.items()}
    write = {k: v[-20:] for k, v in write_all.items()}
    cf, cw = gib / copy_f, gib / copy_w
    kernels = {}
    for k in fetch:
        if "wc::" not in k or k not in write:
            continue
        short = k.replace("void ", "").replace("wc::", "").split("(")[0]
        fb = cf * sum(fetch[k]) / len(fetch[k])
        wb = cw * sum(write[k]) / len(write[k])
        kernels[short] = {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
                          "launches": len(fetch[k])}
    rec = {"csrc_sha256": csrc_sha256(), "fetch_scale": cf, "write_scale": cw,
           "command": "rocprofv3 --pmc FETCH_SIZE|WRITE_SIZE --output-format csv -- python bench.py --profile",
           "kernels": kernels}
    json.dump(rec, open(out_json, "w"), indent=1)
    return rec


def profile_run(wc, torch, dev):
    """A short run for profilers: the 1 GiB calibration copy, two batched 24^3 x 48 solves
    (one warm-up, one measured), then the timing loops of the block solver's half-sweep and
    of D_w (last dispatches of each kernel = the loops bench.py reports)."""
    import synth
    src = torch.ones(128 * 1024 * 1024, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    lat = wc.Lattice(torch.from_numpy(synth.gauge_field(C4_DIMS)).to(dev), block=BLOCK, m0=M0, csw=CSW)
    pts = torch.from_numpy(synth.point_sources(C4_DIMS)).to(dev)
    storage = os.environ.get("WC_BENCH_STORAGE", "bf16")
    basis = os.environ.get("WC_BENCH_BASIS", "f32")
    tiles = lat.autotune(12, prec=storage)
    _TILES[(id(lat), storage)] = tiles[0]
    _TILES[(id(lat), "f64")] = tiles[1]
    p = params(wc, storage, True, basis_prec=basis)
    lat.solve(pts, p)
    (_, st), ms = sync_time(torch, lambda: lat.solve(pts, p))
    rf = roofline_record(lat, 663552, storage, 12, BLOCK, f"k_sap_eo<{storage}, 1 rhs, reloaded>, 24^3x48 x 12 rhs")
    dw = dirac_rates(lat, 663552, ("f64", storage), nrhs=12, iters=20)
    print(json.dumps({"profile": "24^3x48 x 12 point sources", "storage": storage, "basis": basis, "solve_ms": ms,
                      "iters": max(s["iters"] for s in st), "half_sweep_ms": rf["launch_ms"],
                      "dirac_12rhs": dw}), flush=True)


def counter_summary(csv_path, out_md, command, match="k_sap_eo", last=20):
    """Markdown table of a rocprofv3 --pmc run: for each kernel whose name contains `match`,
    the mean of every counter over its last `last` dispatches (the timing loops of
    `bench.py --profile`)."""
    import csv
    rows = [r for r in csv.DictReader(open(csv_path)) if match in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    agg = {}
    for r in rows:
        k = r["Kernel_Name"].replace("void ", "").replace("wc::", "").split("(")[0]
        agg.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    names = sorted({c for d in agg.values() for c in d})
    lines = [f"Command: `{command}`", "", "| kernel | " + " | ".join(names) + " |",
             "|---|" + "---|" * len(names)]
    for k, d in agg.items():
        vals = []
        for c in names:
            v = d.get(c, [])[-last:]
            vals.append(f"{sum(v) / len(v):.6g}" if v else "")
        lines.append(f"| `{k}` | " + " | ".join(vals) + " |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    return {k: {c: sum(v[-last:]) / len(v[-last:]) for c, v in d.items()} for k, d in agg.items()}


def profile_summary(stats_dir, out_md, command, traffic_json=None, top=16):
    """Markdown summary of a rocprofv3 --kernel-trace --stats run of `bench.py --profile`:
    per-kernel calls, mean and total time from the stats CSV, the mean of each kernel's last
    20 dispatches from the trace (the timing loops bench.py reports), and, with a traffic
    record, the HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE passes."""
    import csv
    stats = list(csv.DictReader(open(os.path.join(stats_dir, "run_kernel_stats.csv"))))
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    trace = list(csv.DictReader(open(os.path.join(stats_dir, "run_kernel_trace.csv"))))
    trace.sort(key=lambda r: int(r["Start_Timestamp"]))
    durs = {}
    for r in trace:
        durs.setdefault(r["Kernel_Name"], []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    traffic = json.load(open(traffic_json))["kernels"] if traffic_json else {}
    lines = [f"Command: `{command}`", "", "| kernel | calls | mean us | last 20 mean us | total ms | % | "
             "HBM MB / launch (last 20) |", "|---|---|---|---|---|---|---|"]
    for r in stats[:top]:
        name = r["Name"]
        last = durs.get(name, [])[-20:]
        short = name.replace("void ", "").replace("wc::", "").split("(")[0]
        t = traffic.get(short)
        mb = f"{t['bytes_per_launch'] / 1e6:.1f}" if t else ""
        lines.append(f"| `{short}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{(sum(last) / len(last)) if last else 0.0:.2f} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['Percentage']):.1f} | {mb} |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    return lines


def profile_dirac_run(wc, torch, dev):
    """A short run for profilers of single-rhs D_w at 32^3 x 64 in every storage precision
    (the 1 GiB calibration copy first, then 30 launches per precision); prints the HIP-event
    times and the algorithmic bytes per launch."""
    import synth
    src = torch.ones(128 * 1024 * 1024, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    lat = wc.Lattice(torch.from_numpy(synth.gauge_field(C3_DIMS)).to(dev), block=BLOCK, m0=M0, csw=CSW)
    V = 2097152
    out = {}
    for prec in ("f64", "f32", "f16", "bf16"):
        ms = lat.bench_dirac(prec=prec, nrhs=1, iters=30)
        out[prec] = {"ms": ms, "alg_bytes_per_launch": dw_bytes(prec) * V,
                     "frac_hbm": dw_bytes(prec) * V / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    print(json.dumps({"profile": "D_w 32^3x64, 1 rhs", "dirac": out}), flush=True)


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarise-pmc":
        summarise_pmc(sys.argv[2], sys.argv[3], sys.argv[4])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--valu-record":
        # --valu-record CSV OUT_JSON
        valu_record(sys.argv[2], sys.argv[3])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--counter-summary":
        # --counter-summary CSV OUT_MD COMMAND [MATCH]
        counter_summary(sys.argv[2], sys.argv[3], sys.argv[4], *(sys.argv[5:6]))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--profile-summary":
        # --profile-summary STATS_DIR OUT_MD COMMAND [TRAFFIC_JSON]
        profile_summary(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5] if len(sys.argv) > 5 else None)
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extras", action="store_true", help="only the headline step and its roofline")
    ap.add_argument("--profile", action="store_true", help="short run for profilers (no tuning, no extras)")
    ap.add_argument("--profile-dirac", action="store_true", help="short profiler run of single-rhs D_w at 32^3x64")
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
    if args.profile:
        profile_run(wc, torch, dev)
        return
    if args.profile_dirac:
        profile_dirac_run(wc, torch, dev)
        return
    V = 663552
    lat = wc.Lattice(torch.from_numpy(synth.gauge_field(C4_DIMS)).to(dev), block=BLOCK, m0=M0, csw=CSW)
    pts = torch.from_numpy(synth.point_sources(C4_DIMS)).to(dev)
    # the baseline of the target: 12 single-rhs solves with the plain FP64 method (MR on
    # D_Lambda, 4^4 blocks as configured for the FP64 solver), and FP64 with the even/odd
    # block solver, on the same lattice
    t_mr, it_mr = single_solves(lat, pts, params(wc, "f64", False), torch)
    t_eo, it_eo = single_solves(lat, pts, params(wc, "f64", True), torch)
    tuning = tune_c4(wc, torch, lat, pts)
    storage = tuning["storage"]
    basis = tuning["basis"]
    block = tuple(tuning["block"])
    p = params(wc, storage, True, basis_prec=basis)

    for _ in range(args.warmup):
        lat.solve(pts, p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(args.steps):
        x, st = lat.solve(pts, p)
        stats.append(st)
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    st = stats[-1]
    iters = max(s["iters"] for s in st)
    restarts = max(s["restarts"] for s in st)
    worst = max(s["rel_true_res"] for s in st)
    # the answer checked with the library's FP64 operator, and against independent FP64
    # references (plain MR block solver, tol 1e-12) on sampled right-hand sides
    r = pts - lat.apply_D(x)
    res_check = max((torch.linalg.vector_norm(r[i]) / torch.linalg.vector_norm(pts[i])).item() for i in range(12))
    errs = []
    for i in (0, 7, 11):
        xr, _ = lat.solve(pts[i].contiguous(), params(wc, "f64", False, tol=1e-12))
        errs.append((torch.linalg.vector_norm(x[i] - xr) / torch.linalg.vector_norm(xr)).item())
    del r
    value = 12 / (ms_per_step * 1e-3)
    flops = sum(solve_flops(V, s["iters"], s["restarts"], NKV, NCY, NMR, block, True) for s in st)
    etile = tuning["tiles"][storage][3]
    roofline = roofline_record(lat, V, storage, 12, block,
                               f"k_sap_eo<{storage}, {etile} rhs per work-group, operator reloaded>: one colour "
                               f"of 24^3x48 x 12 rhs, {NMR} steps", tile=etile)
    pcode = {"f32": 1, "f16": 2, "bf16": 3}[storage]
    roofline["traffic"] = measured_traffic(f"k_sap_eo<{pcode}, {etile}, false>", "traffic_24c48.json")
    roofline["valu_occupancy"] = measured_valu(f"k_sap_eo<{pcode}, {etile}, false>", "valu_24c48.json")

    extras = {}
    if not args.no_extras:
        extras = extra_workloads(wc, torch, dev, storage, lat, pts)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(iters, restarts, workers=min(16, host_cores()))

    out = {
        "metric": "D_w GB/s & Gflop/s vs HBM roofline; FGCR time-to-1e-10 (mixed vs FP64)",
        "value": value,
        "unit": "rhs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "batched SAP-FGCR solve of the 12 spin-colour point sources to a true residual "
                               "of 1e-10 each, 24^3x48, eps=0.3 gauge, m0=-0.1, c_sw=1, FP32 Schwarz "
                               f"preconditioner on {storage} storage (even/odd block solver, nmr=4, ncy=5), "
                               f"FGCR (nkv=16) in FP64 arithmetic over an {basis} Krylov basis"
                               + (" (cycles end at a 1e-6 drop; FP64 residual and solution at each restart)"
                                  if basis == "f32" else "") + ", one graph per restart cycle",
                   "lattice": list(C4_DIMS), "block": list(block), "storage": storage, "basis": basis, "rhs": 12,
                   "parallelism": "single GPU"},
        "ms_per_rhs": ms_per_step / 12,
        "speedup_per_rhs_vs_fp64_single_rhs": 12 * t_mr / ms_per_step,
        "speedup_per_rhs_vs_fp64_eo_single_rhs": 12 * t_eo / ms_per_step,
        "fp64_single_rhs": {"ms": t_mr, "iters": it_mr, "method": "FP64 SAP-FGCR, MR on D_Lambda, 4^4 blocks"},
        "fp64_eo_single_rhs": {"ms": t_eo, "iters": it_eo},
        "iters": iters, "restarts": restarts, "max_true_rel_residual": worst,
        "max_true_rel_residual_recomputed": res_check,
        "rel_err_vs_fp64_reference_sampled_rhs": errs,
        "sustained_Gflops_executed": flops / (ms_per_step * 1e-3) / 1e9,
        "tuning": tuning,
        "roofline": roofline,
        "cpu_baseline": cpu,
        **extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
