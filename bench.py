#!/usr/bin/env python3
"""Benchmark: MLUPS and HBM-roofline fraction of the D2Q37 PML stream-collide on one MI355X.

Workload (one "step" = one full time step of the hot path: PML phase A, boundary/PML frame,
bulk stream-collide): 1024^2 bulk + 32-cell PML on every side (1088^2 grid), characteristic
non-reflecting outer boundary, mean flow Mach 0.1 in +x, isentropic vortex (strength 0.05,
radius 16 cells) plus a Gaussian pulse (A = 1e-3, b = 4) at a seeded position in the central
quarter; FP64 storage is the headline line, FP32 and FP16 deviation storage are reported beside
it.  Inputs are synthetic and resident in HBM before timing starts.

Prints ONE JSON line.  --gpus N > 1 exits with a message: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_NODE = {"f64": 592, "f32": 296, "f16": 148}   # 2 x 37 populations, read + write
PML_EXTRA = {"f64": 656, "f32": 328, "f16": 328}        # Q (37) + U (4) read + write


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_run(lbm, wl, storage, stream, alloc, L, W, sigma, mach, bc, layout=0, bulk_tx=64,
             overlap=0):
    spec = wl.vortex_pulse(L=L, W=W, sigma_max=sigma, mach=mach, bc=bc)
    r = lbm.Run(L, L, 0.8, 1.0, mach, 0.0, 1.0, storage=storage, stream=stream, allocator=alloc,
                layout=layout)
    r.set_launch(bulk_tx=bulk_tx, overlap=overlap)
    r.set_bc(lbm.LBM_ALL, bc)
    if W:
        r.set_pml(lbm.LBM_ALL, W, sigma)
    r.init(*spec.fields.as_tuple())
    return r, spec


def time_run(torch, r, steps, warmup, mode):
    """Time `steps` steps after `warmup`.  mode 2: the configured schedule (in order, or with
    the boundary/PML chain on a side stream beside the bulk kernel) with HIP events around each
    bulk launch on its stream.  mode 1: the kernel classes in order, events around each class."""
    r.profile(0)
    r.step(warmup)
    r.synchronize()
    r.profile(mode)
    r.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r.step(steps)
    r.synchronize()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms, n = r.profile_read(reset=True)
    r.profile(0)
    return dt, ms, n


def serve_trace(jobs, rate, scale, storage, tick):
    from paper_2504_20169_amd import workloads as wl
    from paper_2504_20169_amd.serve import Engine, GpuBackend, jobs_from_trace
    trace = wl.poisson_trace(jobs, rate=rate, seed=5)
    be = GpuBackend(storage=storage)
    eng = Engine(be, int(200e9), tick_steps=tick)
    rep = eng.run_trace(jobs_from_trace(trace, scale))
    be.close()
    return rep


def cpu_baseline(wl, L, W, sigma, mach, bc, steps):
    import oracle
    spec = wl.vortex_pulse(L=L, W=W, sigma_max=sigma, mach=mach, bc=bc)
    o = oracle.OracleRun(L, L, 0.8, 1.0, mach, 0.0, 1.0)
    o.set_bc(15, {"zg": 1, "nrbc": 2}[bc])
    if W:
        o.set_pml(15, W, sigma)
    o.init(*spec.fields.as_tuple())
    o.step(1)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    Nx, Ny = o.grid()
    return Nx * Ny * steps / dt / 1e6, oracle.threads(), dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--L", type=int, default=1024)
    ap.add_argument("--W", type=int, default=32)
    ap.add_argument("--sigma", type=float, default=0.0015)
    ap.add_argument("--mach", type=float, default=0.1)
    ap.add_argument("--bc", default="nrbc")
    ap.add_argument("--storages", default="f64,f32,f16")
    ap.add_argument("--layout", type=int, default=0, help="0: row-interleaved, 1: plane per velocity")
    ap.add_argument("--bulk-tx", type=int, default=64, help="bulk tile width (64, 128 or 256)")
    ap.add_argument("--overlap", type=int, default=0,
                    help="1: boundary/PML chain on a side stream beside the bulk kernel")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=300)
    ap.add_argument("--prof-steps", type=int, default=500,
                    help="steps of a separate pass that runs the kernel classes in order and times "
                         "each (0 skips it)")
    ap.add_argument("--serve-jobs", type=int, default=24, help="0 skips the serving trace")
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-scale", type=float, default=0.1,
                    help="multiplier on the trace's step counts (1000-20000)")
    ap.add_argument("--no-copy-bw", dest="copy_bw", action="store_false",
                    help="skip timing a plain 2 GiB device copy (attainable HBM bandwidth)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of 1 GiB (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2504_20169_amd import lbm
    from paper_2504_20169_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(3)
    lbm.load()
    dev = torch.cuda.get_device_properties(0)
    # Runs own their stream (so --overlap 1 can fork the boundary/PML chain onto a side stream)
    # and take device memory from hipMalloc.
    stream = None
    alloc = None

    if args.copy_calibration:
        n = 1 << 30
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    # attainable HBM bandwidth on this device: a plain 2 GiB device copy (read + write bytes)
    copy_gbs = None
    if args.copy_bw:
        n = 1 << 31
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        copy_gbs = 2.0 * n * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del a, b

    results = {}
    for storage in args.storages.split(","):
        _log("bench: storage", storage)
        r, spec = make_run(lbm, wl, storage, stream, alloc, args.L, args.W, args.sigma,
                           args.mach, args.bc, args.layout, args.bulk_tx, args.overlap)
        Nx, Ny = r.grid()
        n_bulk, n_frame, n_q = r.node_classes()
        dt, ms_live, n_live = time_run(torch, r, args.steps, args.warmup, mode=2)
        if args.prof_steps > 0:
            _, ms, n = time_run(torch, r, args.prof_steps, 5, mode=1)
        else:
            ms, n = np.zeros(3), np.zeros(3, dtype=np.int64)
        st = r.check()
        nodes = Nx * Ny
        mlups = nodes * args.steps / dt / 1e6
        alg_bytes_step = BYTES_PER_NODE[storage] * nodes + PML_EXTRA[storage] * n_q
        bulk_ms = ms_live[0] / max(n_live[0], 1)
        bulk_bytes = BYTES_PER_NODE[storage] * n_bulk
        results[storage] = dict(
            mlups=mlups, mlups_bulk=args.L * args.L * args.steps / dt / 1e6,
            ms_per_step=dt * 1e3 / args.steps,
            gbs_step=alg_bytes_step / (dt / args.steps) / 1e9,
            bulk_kernel_ms=bulk_ms,
            bulk_kernel_gbs=bulk_bytes / (bulk_ms * 1e-3) / 1e9 if bulk_ms > 0 else None,
            bulk_nodes=n_bulk, frame_nodes=n_frame, q_nodes=n_q, bulk_bytes_per_launch=bulk_bytes,
            stable=(st == lbm.LBM_OK))
        if args.prof_steps > 0:
            results[storage]["in_order"] = dict(
                steps=args.prof_steps,
                bulk_kernel_ms=ms[0] / max(n[0], 1), frame_kernel_ms=ms[1] / max(n[1], 1),
                phase_a_kernel_ms=ms[2] / max(n[2], 1),
                boundary_cost_ratio=(ms[1] + ms[2]) / max(ms[0], 1e-9),
                ms_per_step=sum(ms) / max(n[1], 1))
        if storage != "f64" and "f64" in results:
            rho_ref, ux_ref, uy_ref, T_ref = results["f64"]["_moments"]
            rho, ux, uy, T = r.moments()
            us = max(np.abs(ux_ref).max(), np.abs(uy_ref).max())
            results[storage]["err_vs_f64"] = dict(
                rho=float(np.abs(rho - rho_ref).max() / np.abs(rho_ref).max()),
                u=float(max(np.abs(ux - ux_ref).max(), np.abs(uy - uy_ref).max()) / us),
                T=float(np.abs(T - T_ref).max() / np.abs(T_ref).max()))
        if storage == "f64":
            results["f64"]["_moments"] = r.moments()
        r.close()
        del r

    main_s = "f64" if "f64" in results else args.storages.split(",")[0]
    R = results[main_s]
    line = {
        "metric": "MLUPS (all grid nodes) and % HBM roofline of the fused PML stream-collide",
        "value": round(R["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(R["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_s,
        "data": "synthetic",
        "config": {
            "workload": "d2q37_vortex_pulse_%dsq_pml%d_%s_mach%.2g" % (args.L, args.W, args.bc, args.mach),
            "bulk": args.L, "pml_width": args.W, "grid": args.L + 2 * args.W, "boundary": args.bc,
            "sigma_max": args.sigma, "tau": 0.8, "storage": main_s, "layout": args.layout,
            "bulk_tx": args.bulk_tx, "overlap": args.overlap,
            "device": dev.name,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_bulk (interior fused stream-collide)",
            "achieved": round(R["bulk_kernel_gbs"], 1) if R["bulk_kernel_gbs"] else None,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(R["bulk_kernel_gbs"] / HBM_PEAK_GBS, 4) if R["bulk_kernel_gbs"] else None,
            "traffic": None,
            "bytes_per_launch": R["bulk_bytes_per_launch"],
            "avg_launch_ms": round(R["bulk_kernel_ms"], 5),
            "device_copy_gbs": round(copy_gbs, 1) if copy_gbs else None,
            "timing": "HIP events around each k_bulk launch on its stream inside the timed %d steps"
                      % args.steps,
        },
        "variants": {},
    }
    def rnd(v):
        if isinstance(v, dict):
            return {k: rnd(x) for k, x in v.items() if not k.startswith("_")}
        return round(v, 6) if isinstance(v, float) else v
    for s, v in results.items():
        line["variants"][s] = rnd(v)
    if args.serve_jobs > 0:
        _log("bench: serving trace")
        line["serving"] = serve_trace(args.serve_jobs, args.serve_rate, args.serve_scale, "f32", 200)
        line["serving"].update(trace="%d Poisson arrivals at %.0f/s, steps x%.2g, FP32 storage, "
                                     "HBM budget 200 GB" % (args.serve_jobs, args.serve_rate, args.serve_scale))
    if not args.no_cpu:
        _log("bench: cpu baseline (oracle)")
        mlups_cpu, cores, dt_cpu = cpu_baseline(wl, args.L, args.W, args.sigma, args.mach, args.bc,
                                                args.cpu_steps)
        line["cpu_baseline"] = {"value": round(mlups_cpu, 2), "unit": "MLUPS", "cores": cores,
                                "kind": "oracle",
                                "sample": "%d steps of the same %d^2 FP64 workload (%.1f s)"
                                          % (args.cpu_steps, args.L + 2 * args.W, dt_cpu)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
