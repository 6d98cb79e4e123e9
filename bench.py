#!/usr/bin/env python3
"""Throughput of the grid-integration step on one MI355X.

One step is the whole hot path on the Si-512 DZP workload (4x4x4 diamond
supercell, atoms displaced N(0, 0.05 bohr), 6656 orbitals, rc = 8 bohr,
192^3 mesh): re-binning of the batch/atom lists for the current positions,
the local-potential matrix H, the density rho and the grid force dE/dR
(the cal_gint_vl + cal_gint_rho + cal_gint_fvl triple that the paper times
per step in its Gint scaling test, Sec. 4.3.1).  Inputs are resident in HBM
before the timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import re
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6  # MI355X dense FP64 matrix peak
PEAK_FP32_TFLOPS = 157.3  # MI355X dense FP32 matrix peak
PEAK_16BIT_TFLOPS = 2500.0  # MI355X dense BF16 / FP16 matrix peak
# arithmetic type of the path per mode: H operands (+ rho/force operands) and accumulation
DTYPES = {"fp64": "f64", "fp32": "f32 (f64 sums)", "bf16": "bf16 H, f32 rho/force (f64 sums)",
          "fp16": "f16 H, f32 rho/force (f64 sums)", "bf16x3": "bf16 hi/lo H, f32 rho/force (f64 sums)",
          "fp16x3": "f16 hi/lo H and rho/force contraction, f32 accumulation (f64 sums)"}
PEAK_HBM_GBS = 8000.0

N_XCD = 8  # MI355X: accelerator complex dies (GRBM_GUI_ACTIVE is summed over them)
N_SIMD = 1024  # 256 compute units x 4 SIMDs


def fused_peak(prec: str, kernel: str):
    """The matrix peak a contraction kernel is priced at, and why."""
    if prec == "fp64":
        return PEAK_FP64_TFLOPS, "FP64 matrix cores"
    if prec == "fp16x3" and kernel in ("H_rho_force", "rho_force", "force", "H_blocks"):
        # every multiply-add of the n_g^2 work runs as three FP16 products
        return PEAK_16BIT_TFLOPS / 3, ("H and T = (D + D^T) phi on FP16 matrix cores, three hi/lo products "
                                       "per multiply-add: the 16-bit peak / 3")
    if kernel == "H_blocks" and prec != "fp32":
        return PEAK_16BIT_TFLOPS, "16-bit matrix cores"
    return PEAK_FP32_TFLOPS, ("T = (D + D^T) phi on FP32 matrix cores (the larger share), H on the mode's; "
                              "priced at the FP32 peak")


def _kernel_sha() -> str:
    h = hashlib.sha256()
    for f in ("gint_kernels.hip", "gint_contract.hip", "gint_device.h", "gint_internal.h"):
        with open(os.path.join(ROOT, "paper_2603_21835_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel: str, workload: str, precision: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_sha") != _kernel_sha():
        return None
    return t.get("bytes_per_launch")


# device kernel (symbol prefix) behind each timing kind whose traffic is recorded
KERNEL_SYMBOLS = {"rho_force": r"k_force_packed<[^>]*, 0, (?:true|false)>",
                  "H_rho_force": r"k_force_packed<[^>]*, [1-6], (?:true|false)>",
                  "H_blocks": r"k_H_batch<", "H_reduce": r"k_H_pairreduce<"}


def _counter_csv(d: str, counter: str):
    """(kernel name, value) per dispatch of one counter from a rocprofv3 --pmc CSV directory."""
    import csv
    import glob

    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    if not rows:
        raise SystemExit(f"no {counter} rows under {d}")
    return rows


def write_traffic(args):
    """HBM bytes per launch of one kernel from FETCH_SIZE / WRITE_SIZE runs
    (KiB per dispatch), each scaled by what the same counter reads for a plain
    copy of known size (the largest copy dispatch of the calibration runs)."""
    d = args.traffic_from
    sym = KERNEL_SYMBOLS[args.kernel]
    with open(os.path.join(d, "copy_bytes.json")) as fh:
        copy_bytes = json.load(fh)["copy_bytes"]
    out = {"kernel": args.kernel, "symbol": sym, "workload": args.workload, "precision": args.precision,
           "kernel_sha": _kernel_sha()}
    total = 0.0
    for name, counter in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        copy_kib = max(v for _, v in _counter_csv(os.path.join(d, "copy_" + name), counter))
        factor = copy_bytes / (copy_kib * 1024.0)
        vals = [v for k, v in _counter_csv(os.path.join(d, name), counter) if re.search(sym, k)]
        if not vals:
            raise SystemExit(f"no {sym} dispatch in {d}/{name}")
        per = sum(vals) / len(vals) * 1024.0 * factor
        out[name] = {"counter": counter, "kib_per_dispatch": sum(vals) / len(vals), "dispatches": len(vals),
                     "copy_kib": copy_kib, "scale": factor, "bytes_per_launch": per}
        total += per
    out["bytes_per_launch"] = total
    path = os.path.join(ROOT, "profiles", f"traffic_{args.kernel}_{args.workload}_{args.precision}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out), flush=True)


def write_mfma(args):
    """Issued FP64 matrix work of one kernel per launch from a rocprofv3 --pmc
    run with SQ_INSTS_VALU_MFMA_MOPS_F64 (one MOP = 512 flops),
    SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE (summed over the 8 XCDs)."""
    d = args.mfma_from
    sym = KERNEL_SYMBOLS[args.kernel]
    vals = {}
    for counter in ("SQ_INSTS_VALU_MFMA_MOPS_F64", "SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE"):
        v = [x for k, x in _counter_csv(d, counter) if re.search(sym, k)]
        if not v:
            raise SystemExit(f"no {sym} dispatch with {counter} in {d}")
        vals[counter] = sum(v) / len(v)
    grbm_xcd = vals["GRBM_GUI_ACTIVE"] / N_XCD
    out = {"kernel": args.kernel, "symbol": sym, "workload": args.workload, "precision": args.precision,
           "kernel_sha": _kernel_sha(), "counters": vals,
           "issued_flops_per_launch": vals["SQ_INSTS_VALU_MFMA_MOPS_F64"] * 512.0,
           "mfma_busy": vals["SQ_VALU_MFMA_BUSY_CYCLES"] / (grbm_xcd * N_SIMD)}
    path = os.path.join(ROOT, "profiles", f"mfma_{args.kernel}_{args.workload}_{args.precision}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out), flush=True)


def _mfma(kernel: str, workload: str, precision: str):
    """Issued matrix flops per launch and the matrix-pipe busy fraction from
    committed counter runs, if they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"mfma_{kernel}_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_sha") != _kernel_sha():
        return None
    return t


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _host_cpu():
    """CPU model and physical core count of this host (from /proc/cpuinfo)."""
    model, cores = "unknown", set()
    try:
        phys = core = None
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and model == "unknown":
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None and core is not None:
                    cores.add((phys, core))
                    phys = core = None
        if phys is not None and core is not None:
            cores.add((phys, core))
    except OSError:
        pass
    return model, len(cores) or None


def cpu_baseline(w):
    """Time the FP64 oracle (as it stands) on a bounded sample of the same
    workload and extrapolate to one full step: H rows and dE/dR of one atom
    per oracle thread (the oracle is parallel over atoms for both) summed
    over a random half of the mesh points, and rho at 40000 mesh points
    (parallel over points): about 10 s of host time.  A single-thread run of
    one atom's H rows and dE/dR over 1/16 of the mesh gives the one-core
    rate (a few seconds)."""
    import oracle

    o = oracle.Oracle.from_workload(w)
    nthr = oracle.num_threads()
    rng = np.random.default_rng(0)
    na = min(w.natom, max(nthr, 1))
    lo = int(rng.integers(0, w.natom - na + 1))
    atoms = np.arange(lo, lo + na, dtype=np.int32)
    npts = min(40000, w.ngrid)
    idx = np.sort(rng.choice(w.ngrid, npts, replace=False))
    nsub = max(1, w.ngrid // 2)
    sub = np.sort(rng.choice(w.ngrid, nsub, replace=False))
    t = time.perf_counter()
    o.H_rows(w.V, lo, lo + na, points=sub)
    tH = time.perf_counter() - t
    t = time.perf_counter()
    o.force(w.V, w.D, atoms, points=sub)
    tF = time.perf_counter() - t
    t = time.perf_counter()
    o.rho(w.D, idx)
    tR = time.perf_counter() - t
    t_step = (tH + tF) * (w.natom / na) * (w.ngrid / nsub) + tR * w.ngrid / npts
    # one thread: H rows and dE/dR of one atom over 1/16 of the mesh
    n1 = max(1, w.ngrid // 16)
    sub1 = np.sort(rng.choice(w.ngrid, n1, replace=False))
    oracle.set_threads(1)
    try:
        t = time.perf_counter()
        o.H_rows(w.V, lo, lo + 1, points=sub1)
        o.force(w.V, w.D, atoms[:1], points=sub1)
        t1 = time.perf_counter() - t
    finally:
        oracle.set_threads(nthr)
    t_step1 = t1 * w.natom * (w.ngrid / n1) + tR * nthr * w.ngrid / npts
    model, phys = _host_cpu()
    return {
        "value": w.ngrid / t_step,
        "unit": "grid pts/s",
        "cores": int(nthr),
        "physical_cores": phys,
        "logical_cpus": os.cpu_count(),
        "cpu_model": model,
        "single_thread_value": w.ngrid / t_step1,
        "kind": "oracle",
        "sample": (f"{w.name}: H rows of atoms {lo}..{lo + na - 1} ({tH:.1f} s) and dE/dR of the same "
                   f"{na} atoms ({tF:.1f} s), both over {nsub} random mesh points; rho at {npts} random "
                   f"mesh points ({tR:.1f} s); "
                   f"extrapolated linearly to all {w.natom} atoms and {w.ngrid} points = "
                   f"{t_step:.0f} s per step on {nthr} threads; one thread: one atom's H rows and dE/dR over "
                   f"{n1} points ({t1:.1f} s), rho as above scaled by {nthr} threads, = {t_step1:.0f} s per step"),
    }


def mixed_leg(args, w, V, D, H64, rho64, F64, torch, g, dev, ms_fp64):
    """The same step (re-binning + gint_H_rho_force) in the FP16 hi/lo mode
    (H and the rho / force contraction on FP16 matrix cores with 3 products,
    FP32 orbital tiles, FP64 sums across batches), timed like the FP64 step, with its
    error against the FP64 GPU outputs of the same inputs."""
    prec = "fp16x3"
    plan = g.GintPlan.from_workload(w, precision=prec)
    H = torch.empty((plan.norb, plan.norb), dtype=torch.float64, device=dev)
    rho = torch.empty(plan.ngrid, dtype=torch.float64, device=dev)
    F = torch.empty((plan.natom, 3), dtype=torch.float64, device=dev)

    def step():
        plan.set_positions(w.positions)
        plan.H_rho_force(V, D, H=H, rho=rho, out=F)

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = plan.timing()
    plan.set_timing(False)
    work = plan.work()
    ms = (t1 - t0) * 1e3 / args.steps
    s1, s2 = work["sum_ng"], work["sum_ng2"]
    kernels = {k: {"avg_ms": round(t / n, 4), "launches": n} for k, (t, n) in timing.items() if n}
    dom = max(kernels, key=lambda k: timing[k][0])
    roof = None
    if dom == "H_rho_force":
        per = (4 * s2 + 8 * s1) / (timing[dom][1] / args.steps)
        ach = per / (kernels[dom]["avg_ms"] * 1e-3) / 1e12
        peak, why = fused_peak(prec, dom)
        roof = {"bound": "mfma", "kernel": dom, "achieved": round(ach, 3), "peak": round(peak, 1),
                "unit": "TFLOP/s", "frac": round(ach / peak, 4), "note": "fused pass: " + why}
    out = {
        "precision": prec,
        "dtype": DTYPES[prec],
        "ms_per_step": ms,
        "value": w.ngrid / (ms * 1e-3),
        "unit": "grid pts/s",
        "speedup_vs_fp64": ms_fp64 / ms,
        "max_abs_dH_Ha": float((H - H64).abs().max()),
        "meets_1e-6_Ha": bool(float((H - H64).abs().max()) <= 1e-6),
        "rho_rel_l2": float(torch.linalg.norm(rho - rho64) / torch.linalg.norm(rho64)),
        "force_rel_max": float((F - F64).abs().max() / F64.abs().max()),
        "error_reference": "the FP64 GPU path on the same inputs (itself within 1e-10 of the FP64 oracle)",
        "roofline": roof,
        "kernels": kernels,
    }
    plan.close()
    return out


def run_batched(args, torch, gi, g, dev):
    """256 independent Si cells of 8..64 atoms: H, rho and dE/dR of every
    cell per step, each quantity one replay of a captured hipGraph.  The
    cells' geometry is fixed across steps (no re-binning in the step)."""
    _progress(f"generating {args.cells} cells")
    cells = gi.batched_cells(args.cells)
    ngrid = sum(c.ngrid for c in cells)
    _progress(f"batch plans ({ngrid} points)")
    b = g.GintBatch(cells, cells[0].species, precision=args.precision)
    V = [torch.from_numpy(c.V).to(dev) for c in cells]
    D = [torch.from_numpy(c.D).to(dev) for c in cells]
    H = [torch.empty((n, n), dtype=torch.float64, device=dev) for n in b.norb]
    rho = [torch.empty(n, dtype=torch.float64, device=dev) for n in b.ngrid]
    F = [torch.empty((n, 3), dtype=torch.float64, device=dev) for n in b.natom]

    def step():
        if args.separate:
            b.build_H(V, out=H)
            b.build_rho(D, out=rho)
            b.force(V, D, out=F)
        else:
            b.H_rho_force(V, D, H=H, rho=rho, out=F)  # one graph replay for all three

    def seq_step():
        for i, p in enumerate(b.cells):
            if args.separate:
                p.build_H(V[i], out=H[i])
                p.build_rho(D[i], out=rho[i])
                p.force(V[i], D[i], out=F[i])
            else:
                p.H_rho_force(V[i], D[i], H=H[i], rho=rho[i], out=F[i])

    _progress(f"warmup {args.warmup}")
    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    _progress(f"timed {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    # the same work as per-cell calls on one stream, for comparison
    seq_step()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    seq_step()
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - t2) * 1e3
    s1 = sum(p.work()["sum_ng"] for p in b.cells)
    s2 = sum(p.work()["sum_ng2"] for p in b.cells)
    # H, rho and dE/dR: with the fused call rho and the force share one
    # contraction T = (D + D^T) phi (4 sum n^2 + 8 sum n); as three calls,
    # three contractions
    alg = (6 * s2 + 8 * s1) if args.separate else (4 * s2 + 8 * s1)
    kinds = np.bincount(gi.batched_kinds(args.cells), minlength=4)
    out = {
        "metric": "gint grid pts/s + MFMA util: FP64 vs mixed precision at stated |dH| (Si-512)",
        "value": ngrid / (ms_step * 1e-3),
        "unit": "grid pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[args.precision],
        "data": "synthetic",
        "config": {
            "workload": (f"{args.cells} independent Si cells (8/16/32/64 atoms: {kinds.tolist()}), DZP rc=8 bohr, "
                         f"{ngrid} mesh points in total; one step = H + rho + dE/dR of every cell, "
                         + ("one graph replay each" if args.separate else
                            "one graph replay of gint_H_rho_force over every cell")
                         + ", fixed geometry"),
            "sequential_ms_per_step": seq_ms,
            "graph_speedup_vs_sequential": seq_ms / ms_step,
            "alg_tflops_whole_step": alg / (ms_step * 1e-3) / 1e12,
        },
    }
    b.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="si512", choices=["si512", "si64", "si8", "batched"])
    ap.add_argument("--cells", type=int, default=256, help="number of cells of the batched workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the FP16 hi/lo leg of the default FP64 line")
    ap.add_argument("--precision", default="fp64", choices=list(DTYPES))
    ap.add_argument("--only", default=None,
                    choices=["H", "rho", "force", "rho_force", "H_rho_force", "HR", "rhoR", "forceR", "DK",
                             "psibeta"],
                    help="time one contraction only (short profiler runs); HR: the lattice-vector blocks "
                         "H(R) for every R of gint_HR_lattice; rhoR: rho from random lattice-vector density "
                         "matrices D(R) over the same R; forceR: dE/dR for those D(R); DK: the moving-basis "
                         "matrix <phi_mu|V|d phi_nu/d tau_K> (gint_build_DK); psibeta: the spherical-grid projector "
                         "overlaps <phi_mu|e^{-iA.r}|beta_p> (110 x 140 points per atom, gint_psibeta_overlap)")
    ap.add_argument("--separate", action="store_true",
                    help="rho and the force as two passes (gint_build_rho + gint_force) instead of gint_rho_force")
    ap.add_argument("--serial", action="store_true",
                    help="H and the rho + force pass as two calls (gint_build_H + gint_rho_force) instead of "
                         "gint_H_rho_force")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB mebibytes (counter calibration)")
    ap.add_argument("--traffic-from", default=None, metavar="DIR",
                    help="write profiles/traffic_<kernel>_<workload>_<precision>.json from the rocprofv3 "
                         "counter CSVs under DIR (fetch/, write/, copy_fetch/, copy_write/) and exit")
    ap.add_argument("--mfma-from", default=None, metavar="DIR",
                    help="write profiles/mfma_<kernel>_<workload>_<precision>.json from a rocprofv3 counter CSV "
                         "directory with SQ_INSTS_VALU_MFMA_MOPS_F64, SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE "
                         "and exit")
    ap.add_argument("--kernel", default="rho_force",
                    help="timing kind whose traffic (--traffic-from) or matrix work (--mfma-from) is recorded")
    args = ap.parse_args()
    if args.traffic_from:
        write_traffic(args)
        return
    if args.mfma_from:
        write_mfma(args)
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the multi-GPU "
              f"sharding of this path is a design note, not a built path).", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs as a single process on one GPU.", file=sys.stderr)
        sys.exit(2)

    import torch

    import gint_inputs as gi
    import paper_2603_21835_amd as g

    assert torch.cuda.is_available(), "no GPU visible"
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 8 * n, "launches": 3}), flush=True)
        return
    g.load_library()
    dev = torch.device("cuda:0")
    if args.workload == "batched":
        print(json.dumps(run_batched(args, torch, gi, g, dev)), flush=True)
        return
    _progress(f"generating {args.workload}")
    w = {"si512": gi.si512_dzp, "si64": gi.si64_dzp, "si8": gi.si8_sz}[args.workload]()
    _progress("plan")

    plan = g.GintPlan.from_workload(w, precision=args.precision)
    V = torch.from_numpy(w.V).to(dev)
    D = torch.from_numpy(w.D).to(dev)
    H = torch.empty((plan.norb, plan.norb), dtype=torch.float64, device=dev)
    rho = torch.empty(plan.ngrid, dtype=torch.float64, device=dev)
    F = torch.empty((plan.natom, 3), dtype=torch.float64, device=dev)
    work = plan.work()
    if args.only in ("HR", "rhoR", "forceR"):
        R_list = plan.HR_lattice()
    if args.only == "HR":
        HRbuf = torch.empty((len(R_list), plan.norb, plan.norb), dtype=torch.float64, device=dev)
    if args.only in ("rhoR", "forceR"):
        gen = torch.Generator(device=dev)
        gen.manual_seed(12)
        DRbuf = torch.randn((len(R_list), plan.norb, plan.norb), dtype=torch.float64, device=dev,
                            generator=gen) / plan.norb

    if args.only == "DK":
        DKbuf = torch.empty((3, plan.norb, plan.norb), dtype=torch.float64, device=dev)
    if args.only == "psibeta":
        proj = [gi.si_projector_species()]
        ang, rq = gi.lebedev_110(), gi.gauss_legendre_01(140)
        pb = g.GintPsiBeta(plan, proj, ang, rq)
        Apot = gi.vector_potential(13, 0.05)
        Qbuf = torch.empty((pb.nproj, plan.norb), dtype=torch.complex128, device=dev)

    def step():
        if args.only == "psibeta":
            pb.overlap(Apot, out=Qbuf)
            return
        if args.only == "DK":
            plan.build_DK(V, out=DKbuf)
            return
        if args.only == "HR":
            plan.build_HR(V, R_list, out=HRbuf)
            return
        if args.only == "rhoR":
            plan.build_rhoR(R_list, DRbuf, out=rho)
            return
        if args.only == "forceR":
            plan.forceR(V, R_list, DRbuf, out=F)
            return
        if args.only is None:
            plan.set_positions(w.positions)
        if (args.only is None and not args.serial and not args.separate) or args.only == "H_rho_force":
            plan.H_rho_force(V, D, H=H, rho=rho, out=F)  # H, rho and dE/dR in one call
            return
        if args.only in (None, "H"):
            plan.build_H(V, out=H)
        if (args.only is None and not args.separate) or args.only == "rho_force":
            plan.rho_force(V, D, rho=rho, out=F)  # rho from the force pass
        else:
            if args.only in (None, "rho"):
                plan.build_rho(D, out=rho)
            if args.only in (None, "force"):
                plan.force(V, D, out=F)

    _progress(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    _progress(f"timed {args.steps} steps")
    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = plan.timing()
    plan.set_timing(False)

    ms_step = (t1 - t0) * 1e3 / args.steps
    value = w.ngrid / ((t1 - t0) / args.steps)

    s1, s2 = work["sum_ng"], work["sum_ng2"]
    # algorithmic work per step (per unit: one mesh point with n_g orbitals)
    flops = {"H_blocks": 2 * s2, "rho": 2 * s2 + 2 * s1, "force": 2 * s2 + 6 * s1,
             "rho_force": 2 * s2 + 8 * s1, "H_rho_force": 4 * s2 + 8 * s1, "HR": 2 * s2,
             # three non-symmetric products phi (d_c phi)^T over the supported orbitals
             "DK": 6 * s2}
    if args.only == "psibeta":
        # the contraction over quadrature points of every projector against
        # every orbital of the atoms whose cutoff reaches the projector sphere
        # (complex: 4 flops per multiply-add)
        rb = max(r.rc for r in proj[0].radials)
        rcJ = max(r.rc for r in w.species[0].radials)
        pos = w.positions
        shifts = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)]) @ w.lattice
        near = 0
        for I in range(w.natom):
            d = pos[I][None, None, :] - pos[None, :, :] - shifts[:, None, :]
            near += int(np.any(np.linalg.norm(d, axis=2) < rb + rcJ, axis=0).sum())
        flops["psibeta"] = 4.0 * len(ang) * len(rq) * proj[0].norb * near * w.species[0].norb
        work["psibeta_pairs"] = near
    # the H reduction moves every block partial once and writes H's blocks
    hbytes = {"H_reduce": work["nblock"] * work["mno"] ** 2 * work["partial_bytes"],
              "H_fill": 8 * plan.norb ** 2 * (len(R_list) if args.only == "HR" else 1)}
    if args.only == "HR":
        work_hr = plan.work()
        if work_hr["nblock_hr"] > 0:
            # the fixed-order H(R) reduction moves every unfolded block partial once
            hbytes["HR"] = work_hr["nblock_hr"] * work["mno"] ** 2 * work["partial_bytes"]
            flops.pop("HR")
            work["nblock_hr"] = work_hr["nblock_hr"]
    kernels = {}
    for k, (ms, n) in timing.items():
        if n == 0:
            continue
        per_step = n // args.steps if n % args.steps == 0 else n / args.steps
        kernels[k] = {"avg_ms": round(ms / n, 4), "launches": n, "ms_per_step": round(ms / args.steps, 4)}
        if k in flops:
            kernels[k]["alg_tflops"] = round(flops[k] / (ms / args.steps * 1e-3) / 1e12, 3)
        if k in hbytes:
            kernels[k]["alg_gbs"] = round(hbytes[k] / (ms / args.steps * 1e-3) / 1e9, 1)
        kernels[k]["launches_per_step"] = per_step
    dom = max(kernels, key=lambda k: timing[k][0])
    roof = None
    if dom in flops or dom in hbytes:
        lps = timing[dom][1] / args.steps
        avg_s = kernels[dom]["avg_ms"] * 1e-3
        if dom in flops:
            peak, _ = fused_peak(args.precision, dom)
            per_launch = flops[dom] / lps
            ach = per_launch / avg_s / 1e12
            roof = {"bound": "mfma", "achieved": round(ach, 3), "peak": round(peak, 1), "unit": "TFLOP/s",
                    "frac": round(ach / peak, 4), "kernel": dom, "alg_flops_per_launch": per_launch}
        else:
            per_launch = hbytes[dom] / lps
            ach = per_launch / avg_s / 1e9
            roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(ach / PEAK_HBM_GBS, 4), "kernel": dom, "alg_bytes_per_launch": per_launch}
        roof["traffic"] = _traffic(dom, args.workload, args.precision)
        mf = _mfma(dom, args.workload, args.precision) if args.precision == "fp64" else None
        if mf is not None:
            # matrix work as issued (padded tiles included) over the live launch time
            iss = mf["issued_flops_per_launch"] / avg_s / 1e12
            roof["issued"] = {"achieved": round(iss, 3), "frac": round(iss / PEAK_FP64_TFLOPS, 4),
                              "flops_per_launch": mf["issued_flops_per_launch"],
                              "mfma_busy_counter": round(mf["mfma_busy"], 4)}
        else:
            roof["issued"] = None

    # full-size consistency check: dV sum V rho == Tr(D H)  (adjoint identity)
    check = None
    if args.only is None:
        E1 = plan.dV * float(torch.dot(V, rho))
        E2 = float(torch.sum(D * H))
        check = abs(E1 - E2) / max(abs(E2), 1e-300)

    out = {
        "metric": "gint grid pts/s + MFMA util: FP64 vs mixed precision at stated |dH| (Si-512)",
        "value": value,
        "unit": "grid pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[args.precision],
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: {w.natom} atoms, {plan.norb} orbitals, mesh {'x'.join(map(str, w.grid))}, "
                        "DZP rc=8 bohr, one step = re-binning + H + rho + dE/dR"
                        + (" (H, rho and dE/dR as three passes)" if args.separate else
                           " (H, then rho from the force pass)" if args.serial else
                           " (gint_H_rho_force: one pass per batch for H, rho and dE/dR)"),
            "batch": list(work["batch"]), "h_slabs": work["nslab"], "group_pairs": work["npair"],
            "sum_ng2": s2, "sum_ng": s1,
        },
        "roofline": roof,
        "kernels": kernels,
        "check_E_equals_trDH": check,
    }
    if args.precision != "fp64" and args.only is None:
        # accuracy of the mixed mode at full size, against the FP64 path
        _progress("FP64 reference for the mixed-precision error")
        ref = g.GintPlan.from_workload(w, precision="fp64")
        H64 = ref.build_H(V)
        rho64 = ref.build_rho(D)
        F64 = ref.force(V, D)
        torch.cuda.synchronize()
        out["mixed_error_vs_fp64"] = {
            "max_abs_dH_Ha": float((H - H64).abs().max()),
            "rho_rel_l2": float(torch.linalg.norm(rho - rho64) / torch.linalg.norm(rho64)),
            "force_rel_max": float((F - F64).abs().max() / F64.abs().max()),
        }
        ref.close()
    if args.precision == "fp64" and args.only is None and not args.no_mixed and not args.serial \
            and not args.separate:
        _progress("mixed-precision leg (fp16x3)")
        H64, rho64, F64 = H.clone(), rho.clone(), F.clone()
        plan.close()
        out["mixed_fp16x3"] = mixed_leg(args, w, V, D, H64, rho64, F64, torch, g, dev, ms_step)
        del H64, rho64, F64
    if args.only is not None:
        out["only"] = args.only
    if args.only == "HR":
        out["config"]["workload"] = (f"{w.name}: {w.natom} atoms, {plan.norb} orbitals, mesh "
                                     f"{'x'.join(map(str, w.grid))}, DZP rc=8 bohr, one step = the lattice-vector "
                                     f"blocks H(R) of {len(R_list)} lattice vectors (gint_build_HR)")
        out["config"]["n_R"] = len(R_list)
    if args.only == "psibeta":
        out["config"]["workload"] = (f"{w.name}: {w.natom} atoms x 9 synthetic projectors (l = 0, 1, 2), "
                                     f"{plan.norb} orbitals, one step = <phi_mu|e^{{-iA.r}}|beta_p> on the "
                                     "110-point Lebedev x 140-point Gauss-Legendre grid of every atom "
                                     "(gint_psibeta_overlap)")
        out["config"]["projector_atom_pairs"] = work["psibeta_pairs"]
    if args.only == "DK":
        out["config"]["workload"] = (f"{w.name}: {w.natom} atoms, {plan.norb} orbitals, mesh "
                                     f"{'x'.join(map(str, w.grid))}, DZP rc=8 bohr, one step = the moving-basis "
                                     "matrix DK[c][mu][nu] = <phi_mu|V|d phi_nu/d tau_K> (gint_build_DK)")
    if args.only in ("rhoR", "forceR"):
        what = "rho" if args.only == "rhoR" else "dE/dR"
        call = "gint_build_rhoR" if args.only == "rhoR" else "gint_forceR"
        out["config"]["workload"] = (f"{w.name}: {w.natom} atoms, {plan.norb} orbitals, mesh "
                                     f"{'x'.join(map(str, w.grid))}, DZP rc=8 bohr, one step = {what} from random "
                                     f"density-matrix blocks D(R) of {len(R_list)} lattice vectors ({call})")
        out["config"]["n_R"] = len(R_list)
    if not args.no_cpu_baseline and args.only is None:
        _progress("cpu baseline (oracle sample)")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
