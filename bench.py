#!/usr/bin/env python3
"""Benchmark: MLUPS and HBM-roofline fraction of the D2Q37 PML stream-collide on one MI355X.

Workload (one "step" = one full time step of the hot path: PML phase A, boundary/PML frame,
bulk stream-collide): 1024^2 bulk + 32-cell PML on every side (1088^2 grid), characteristic
non-reflecting outer boundary, mean flow Mach 0.1 in +x, isentropic vortex (strength 0.05,
radius 16 cells) plus a Gaussian pulse (A = 1e-3, b = 4) at a seeded position in the central
quarter; FP64 storage is the headline line, FP32 and FP16 deviation storage are reported beside
it, and the same workloads run again on the D2Q17 stencil.  Inputs are synthetic and resident in
HBM before timing starts.

Prints ONE JSON line.  --gpus N > 1 exits with a message: the library runs on one GPU.
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
ELEM = {"f64": 8, "f32": 4, "f16": 2}       # bytes per stored population
COMPUTE = {"f64": 8, "f32": 4, "f16": 4}    # bytes per Q entry (compute precision)


def bytes_per_node(storage, q=37):
    """Algorithmic bytes of one node update: q populations read and q written."""
    return 2 * q * ELEM[storage]


def pml_extra(storage, q=37):
    """Extra bytes of a PML Q-region node: Q (q entries) and U (4 doubles) read and written."""
    return 2 * q * COMPUTE[storage] + 2 * 4 * 8


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_from_spec(lbm, spec, storage, stream=None, alloc=None, layout=0, bulk_tx=64, overlap=2):
    r = lbm.Run(spec.Lx, spec.Ly, spec.tau, spec.rho0, spec.ux0, spec.uy0, spec.T0, storage=storage,
                stream=stream, allocator=alloc, layout=layout, lattice=spec.lattice)
    r.set_launch(bulk_tx=bulk_tx, overlap=overlap)
    r.set_bc(lbm.LBM_ALL, spec.bc)
    if spec.W:
        r.set_pml(lbm.LBM_ALL, spec.W, spec.sigma_max)
    r.init(*spec.fields.as_tuple())
    return r


def time_run(torch, r, steps, warmup, mode):
    """Time `steps` steps after `warmup`.  mode 3: the configured schedule with HIP events attached
    to the dispatch of the step grid (the fused phase-A + bulk grid, or the bulk kernel) and of
    the frame kernel on every fourth step (a sampled average; the other steps carry no events).
    mode 1: the kernel classes in order, events on each class."""
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


def serve_trace(jobs, rate, scale, storage, tick, seed=5):
    """The serving trace: Poisson arrivals at `rate` jobs/s (seed 5: the trace's stated seed), bulk
    128^2..2048^2 log-uniform, PML 8..64, 1000..20000 steps (times `scale`), ZG or NRBC, FP32
    storage, 200 GB HBM budget; latency from arrival to result on the host."""
    from paper_2504_20169_amd import workloads as wl
    from paper_2504_20169_amd.serve import Engine, GpuBackend, jobs_from_trace
    trace = wl.poisson_trace(jobs, rate=rate, seed=seed)
    be = GpuBackend(storage=storage)
    eng = Engine(be, int(200e9), tick_steps=tick)
    rep = eng.run_trace(jobs_from_trace(trace, scale))
    be.close()
    rep.update(trace="%d Poisson arrivals at %g/s, steps x%g, FP32 storage, HBM budget 200 GB, "
                     "tick %d steps" % (jobs, rate, scale, tick))
    return rep


def kernel_bytes(storage, q, n_bulk, n_frame, n_q, fused=True):
    """Algorithmic bytes per launch of the step grid and of the frame kernel, and per step.
    Per step the method moves 2 q b per node and, on the nodes carrying Q, Q and U read and
    written.  In the fused schedule the step grid holds the bulk tiles (2 q b per interior node)
    and phase A, whose algorithmic share is the Q update: Q^n read, Q^{n+1} written and U^n read
    per Q-region node.  The frame kernel moves 2 q b per frame node and writes U^{n+1} of the Q
    region.  The rest of what the two kernels move is not algorithmic: phase A's pull of the
    populations (the frame kernel pulls them again), the frame kernel's reads of Q^{n+1}, and the
    ring's fill store and read."""
    b2 = bytes_per_node(storage, q)
    step = b2 * (n_bulk + n_frame) + pml_extra(storage, q) * n_q
    grid = b2 * n_bulk + ((pml_extra(storage, q) - 32) * n_q if fused else 0)
    return grid, step - grid, step


def measure(torch, lbm, r, spec, storage, steps, warmup, prof_steps, fused=True):
    """Timed pass (the configured schedule, HIP events on a sample of steps) and, if prof_steps,
    an in-order pass with per-class events.  Returns the result dict of one run."""
    Nx, Ny = r.grid()
    n_bulk, n_frame, n_q, n_ring = r.node_classes()
    dt, ms_live, n_live = time_run(torch, r, steps, warmup, mode=3)
    st = r.check()
    nodes = Nx * Ny
    q = spec.lattice
    grid_bytes, frame_bytes, step_bytes = kernel_bytes(storage, q, n_bulk, n_frame, n_q, fused)
    grid_ms = ms_live[0] / max(n_live[0], 1)
    frame_ms = ms_live[1] / max(n_live[1], 1)
    res = dict(
        mlups=nodes * steps / dt / 1e6, mlups_bulk=spec.Lx * spec.Ly * steps / dt / 1e6,
        ms_per_step=dt * 1e3 / steps,
        gbs_step=step_bytes / (dt / steps) / 1e9,
        frac_step=step_bytes / (dt / steps) / 1e9 / HBM_PEAK_GBS,
        grid_kernel_ms=grid_ms,
        grid_gbs=grid_bytes / (grid_ms * 1e-3) / 1e9 if grid_ms > 0 else None,
        grid_bytes_per_launch=grid_bytes,
        frame_kernel_ms=frame_ms,
        frame_gbs=frame_bytes / (frame_ms * 1e-3) / 1e9 if frame_ms > 0 else None,
        frame_bytes_per_launch=frame_bytes,
        bulk_nodes=n_bulk, frame_nodes=n_frame, q_nodes=n_q, ring_nodes=n_ring,
        launches_timed=int(n_live[0]),
        steps=steps, stable=(st == lbm.LBM_OK))
    if res["grid_gbs"]:
        res["grid_frac"] = res["grid_gbs"] / HBM_PEAK_GBS
    if res["frame_gbs"]:
        res["frame_frac"] = res["frame_gbs"] / HBM_PEAK_GBS
    if prof_steps > 0:
        _, ms, n = time_run(torch, r, prof_steps, 5, mode=1)
        res["in_order"] = dict(
            steps=prof_steps,
            bulk_kernel_ms=ms[0] / max(n[0], 1), frame_kernel_ms=ms[1] / max(n[1], 1),
            phase_a_kernel_ms=ms[2] / max(n[2], 1),
            boundary_cost_ratio=(ms[1] + ms[2]) / max(ms[0], 1e-9),
            ms_per_step=sum(ms) / max(n[1], 1))
    return res


def moment_errors(m, ref):
    """Largest relative differences of the moments (rho, ux, uy, T) from a reference: rho and T
    relative to their largest value, u to the largest velocity component of the reference."""
    rho, ux, uy, T = m
    rho_ref, ux_ref, uy_ref, T_ref = ref
    us = max(np.abs(ux_ref).max(), np.abs(uy_ref).max())
    return dict(rho=float(np.abs(rho - rho_ref).max() / np.abs(rho_ref).max()),
                u=float(max(np.abs(ux - ux_ref).max(), np.abs(uy - uy_ref).max()) / us),
                T=float(np.abs(T - T_ref).max() / np.abs(T_ref).max()))


def _leg_prof(args, steps):
    """Steps of a leg's in-order pass with per-class events: half its timed steps, none when
    --prof-steps is 0 (profiled runs then hold the timed schedule only)."""
    return 0 if args.prof_steps == 0 else steps // 2


def large_leg(torch, lbm, wl, args):
    """4096^2 bulk + 64-cell PML (4224^2 nodes), Mach 0.05, 8 seeded pulses, ZG and NRBC, every
    storage: the largest configuration, where the grid is far larger than the caches."""
    out = {}
    for bc in args.large_bcs.split(","):
        spec = wl.multi_pulse(L=4096, W=64, sigma_max=0.01, mach=0.05, bc=bc)
        ref = None
        for storage in args.storages.split(","):
            _log("bench: 4224^2", bc, storage)
            r = run_from_spec(lbm, spec, storage, layout=args.layout, bulk_tx=args.bulk_tx,
                              overlap=args.overlap)
            res = measure(torch, lbm, r, spec, storage, args.large_steps, 20,
                          _leg_prof(args, args.large_steps), args.overlap == 2)
            if args.large_error_steps > 0:
                # every storage continues to the same step count; FP32 and FP16 are compared with
                # FP64 there (the FP64 path itself is held to the oracle by the parity tests)
                left = args.large_error_steps - r.step_count
                if left > 0:
                    r.step(left)
                m = r.moments()
                res["error_steps"] = r.step_count
                if storage == "f64":
                    ref = m
                elif ref is not None:
                    res["err_vs_f64"] = moment_errors(m, ref)
                del m
            out["%s_%s" % (bc, storage)] = res
            r.close()
            del r
        del ref
    return out


def d2q9_leg(torch, lbm, wl, args):
    """The 1024^2 + 32 PML (1088^2) vortex + pulse with NRBC on the D2Q9 stencil (Sec. 2;
    eq. feq-2), 9 populations per node, in every storage."""
    out = {}
    spec = wl.vortex_pulse(L=args.L, W=args.W, sigma_max=args.sigma, mach=args.mach, bc=args.bc)
    spec.lattice = 9
    for storage in args.storages.split(","):
        _log("bench: d2q9 1088^2", storage)
        r = run_from_spec(lbm, spec, storage, layout=args.layout, bulk_tx=args.bulk_tx,
                          overlap=args.overlap)
        out["%dsq_%s_%s" % (spec.Nx, args.bc, storage)] = measure(
            torch, lbm, r, spec, storage, args.d2q9_steps, args.warmup, _leg_prof(args, args.d2q9_steps),
            args.overlap == 2)
        r.close()
        del r
    return out


def d2q17_leg(torch, lbm, wl, args):
    """The same workloads on the D2Q17 stencil (Sec. 2; eq. feq-3), 17 populations per node:
    1024^2 + 32 PML (1088^2) vortex + pulse with NRBC in every storage, and 4096^2 + 64 PML
    (4224^2) pulses with ZG in FP64 and FP32, where the grid is far larger than the caches."""
    out = {}
    spec = wl.vortex_pulse(L=args.L, W=args.W, sigma_max=args.sigma, mach=args.mach, bc=args.bc)
    spec.lattice = 17
    for storage in args.storages.split(","):
        _log("bench: d2q17 1088^2", storage)
        r = run_from_spec(lbm, spec, storage, layout=args.layout, bulk_tx=args.bulk_tx,
                          overlap=args.overlap)
        out["%dsq_%s_%s" % (spec.Nx, args.bc, storage)] = measure(
            torch, lbm, r, spec, storage, args.d2q17_steps, args.warmup, _leg_prof(args, args.d2q17_steps),
            args.overlap == 2)
        r.close()
        del r
    if args.large_steps > 0:
        big = wl.multi_pulse(L=4096, W=64, sigma_max=0.01, mach=0.05, bc="zg")
        big.lattice = 17
        for storage in ("f64", "f32"):
            _log("bench: d2q17 4224^2", storage)
            r = run_from_spec(lbm, big, storage, layout=args.layout, bulk_tx=args.bulk_tx,
                              overlap=args.overlap)
            out["4224sq_zg_%s" % storage] = measure(torch, lbm, r, big, storage, args.large_steps,
                                                   20, _leg_prof(args, args.large_steps), args.overlap == 2)
            r.close()
            del r
    return out


def batch_leg(torch, lbm, wl, args):
    """256 uneven FP32 runs (bulk 128..1024, PML 0..32, ZG or NRBC): each run stepped alone with
    lbm_step, one run after another (the plain single-run path), then all of them in one group
    (one launch per kernel class and step for the whole batch, replayed from a HIP graph)."""
    specs = wl.batch_sweep(nruns=args.batch_runs, steps=args.batch_steps, sigma_max=0.0015)
    runs = [run_from_spec(lbm, sp, "f32") for sp in specs]
    updates = sum(sp.Nx * sp.Ny for sp in specs) * args.batch_steps
    # algorithmic bytes of one step of every run (2 q b per node, Q and U on the Q region)
    step_bytes = 0
    for r, sp in zip(runs, specs):
        n_bulk, n_frame, n_q, _ = r.node_classes()
        step_bytes += kernel_bytes("f32", sp.lattice, n_bulk, n_frame, n_q)[2]
    for r in runs:
        r.step(2)
    for r in runs:
        r.synchronize()
    t0 = time.perf_counter()
    for r in runs:                  # the plain single-run path: one run at a time
        r.step(args.batch_steps)
        r.synchronize()
    t_seq = time.perf_counter() - t0
    g = lbm.Group()
    for r in runs:
        g.add(r)
    tuned = g.autotune(steps=4)
    g.step(nsteps=2)
    g.synchronize()
    t0 = time.perf_counter()
    g.step(nsteps=args.batch_steps)
    g.synchronize()
    t_grp = time.perf_counter() - t0
    ok = all(r.check() == lbm.LBM_OK for r in runs)
    g.close()
    for r in runs:
        r.close()
    return dict(runs=len(specs), steps=args.batch_steps, nodes=sum(sp.Nx * sp.Ny for sp in specs),
                sequential_mlups=updates / t_seq / 1e6, group_mlups=updates / t_grp / 1e6,
                speedup=t_seq / t_grp, stable=ok, group_launch=tuned,
                step_bytes=step_bytes,
                group_gbs=step_bytes * args.batch_steps / t_grp / 1e9,
                group_frac=step_bytes * args.batch_steps / t_grp / 1e9 / HBM_PEAK_GBS,
                workload="batch sweep: bulk L in {128,256,512,1024}, W in {0,4,8,16,32}, ZG/NRBC, "
                         "vortex + pulse, sigma_max 0.0015, FP32 storage")


KERNEL_SRC = [os.path.join(ROOT, "paper_2504_20169_amd", "csrc", n)
              for n in ("lbm_kernels.hip", "lbm_capi.hip", "lbm_internal.h", "lbm_lattice.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_f64_1088sq_nrbc_pmc.txt")
# the FP64 D2Q37 kernels whose HBM traffic the counter summary records, by short name
TRACKED = {
    "grid": "void lbm::k37::k_phase_a_bulk<double, 64>(lbm::RunDev* const*, int const*, int, int const*, int, int, int, int)",
    "frame": "void lbm::k37::k_frame<double>(lbm::RunDev* const*, int const*, int, int)",
    "bulk": "void lbm::k37::k_bulk<double, 64>(lbm::RunDev* const*, int const*, int, int)",
}
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def kernel_source_hash():
    """Hash of the kernel sources and of the runtime that lays out their data."""
    import hashlib
    h = hashlib.sha256()
    for p in KERNEL_SRC:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def pmc_means(path, counter):
    """Mean counter value (KiB per dispatch) per kernel name from a rocprofv3 --pmc CSV."""
    import csv
    acc = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] != counter:
                continue
            acc.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return acc


def pmc_summary(fetch_csv, write_csv, out_path, command):
    """Text summary of two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE): per-kernel KiB per
    dispatch, the scale factors from the 1 GiB device copy of --copy-calibration, and the HBM
    bytes per launch of the tracked FP64 kernels (the roofline's `traffic`)."""
    fetch, write = pmc_means(fetch_csv, "FETCH_SIZE"), pmc_means(write_csv, "WRITE_SIZE")
    gib_kib = float(1 << 20)
    cf = [v for v in fetch.get(COPY_KERNEL, []) if v > 0.25 * gib_kib]
    cw = [v for v in write.get(COPY_KERNEL, []) if v > 0.5 * gib_kib]
    if not cf or not cw:
        raise SystemExit("no 1 GiB copy dispatch in the counter files (run with --copy-calibration)")
    sf = gib_kib / (sum(cf) / len(cf))
    sw = gib_kib / (sum(cw) / len(cw))
    lines = ["# HBM traffic per dispatch, rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE (two passes)",
             "command: " + command,
             "kernel_source_sha256: " + kernel_source_hash(),
             "copy_calibration: 1 GiB device copy reads FETCH_SIZE %.1f KiB, WRITE_SIZE %.1f KiB"
             % (sum(cf) / len(cf), sum(cw) / len(cw)),
             "scale: fetch x%.4f, write x%.4f" % (sf, sw), "",
             "%-72s %8s %14s %14s %14s" % ("kernel", "n", "FETCH KiB", "WRITE KiB", "scaled MB")]
    for k in sorted(set(fetch) & set(write)):
        f = sum(fetch[k]) / len(fetch[k])
        w = sum(write[k]) / len(write[k])
        lines.append("%-72s %8d %14.1f %14.1f %14.2f" % (k[:72], len(fetch[k]), f, w,
                                                           (f * sf + w * sw) * 1024 / 1e6))
    lines.append("")
    for short, name in TRACKED.items():
        if name in fetch and name in write:
            f = sum(fetch[name]) / len(fetch[name]) * sf * 1024
            w = sum(write[name]) / len(write[name]) * sw * 1024
            lines += ["traffic_%s_bytes_per_launch: %d" % (short, round(f + w)),
                      "traffic_%s_read_bytes: %d" % (short, round(f)),
                      "traffic_%s_write_bytes: %d" % (short, round(w))]
    with open(out_path, "w") as fo:
        fo.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def stats_summary(stats_csv, out_path, command, note):
    """Text summary of a rocprofv3 --kernel-trace --stats run: calls and average / min / max
    dispatch duration per kernel, from its kernel_stats CSV, or from its kernel_trace CSV per
    kernel and grid size (so the workloads of one run that share a kernel stay apart)."""
    import csv
    with open(stats_csv) as f:
        rows = list(csv.DictReader(f))
    lines = ["# rocprofv3 --kernel-trace --stats: per-kernel dispatch durations",
             "command: " + command, note, ""]
    if rows and "Start_Timestamp" in rows[0]:
        acc = {}
        for r in rows:
            if r.get("Kind", "KERNEL_DISPATCH") != "KERNEL_DISPATCH":
                continue
            d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            acc.setdefault((r["Kernel_Name"], int(r["Grid_Size_X"])), []).append(d)
        total = sum(sum(v) for v in acc.values())
        lines.append("%-64s %10s %7s %12s %12s %12s %8s" % ("kernel", "grid", "calls", "avg_us",
                                                          "min_us", "max_us", "pct"))
        for (name, grid), v in sorted(acc.items(), key=lambda kv: -sum(kv[1])):
            lines.append("%-64s %10d %7d %12.2f %12.2f %12.2f %8.2f" % (
                name[:64], grid, len(v), sum(v) / len(v), min(v), max(v), 100.0 * sum(v) / total))
    else:
        lines.append("%-72s %7s %12s %12s %12s %8s" % ("kernel", "calls", "avg_us", "min_us",
                                                     "max_us", "pct"))
        for r in rows:
            lines.append("%-72s %7s %12.2f %12.2f %12.2f %8.2f" % (
                r["Name"][:72], r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
                float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    with open(out_path, "w") as fo:
        fo.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def gaps_summary(trace_csv, out_path, command, note, kernel="k_frame", steps=200):
    """Idle time between kernel dispatches in a rocprofv3 --kernel-trace CSV, over the last
    `steps` dispatches of `kernel` at its largest grid (the steps of the timed run: a group's
    launches are the largest): the window runs from the end of the dispatch of `kernel` before
    them to the end of the last, and busy time is the union of the dispatch intervals inside it.
    The idle part is what a persistent kernel that replaces the launches could recover at most."""
    import csv
    with open(trace_csv) as f:
        rows = [r for r in csv.DictReader(f) if r.get("Kind", "KERNEL_DISPATCH") == "KERNEL_DISPATCH"]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    ks = [r for r in rows if kernel in r["Kernel_Name"]]
    gmax = max(int(r["Grid_Size_X"]) for r in ks)
    ks = [r for r in ks if int(r["Grid_Size_X"]) == gmax]
    if len(ks) < steps + 1:
        raise SystemExit("only %d dispatches of %s at grid %d" % (len(ks), kernel, gmax))
    t0, t1 = int(ks[-steps - 1]["End_Timestamp"]), int(ks[-1]["End_Timestamp"])
    inside = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]) for r in rows
              if int(r["Start_Timestamp"]) >= t0 and int(r["End_Timestamp"]) <= t1]
    busy, cur_s, cur_e = 0, None, None
    per = {}
    for a, e, name in inside:
        per.setdefault(name, []).append(e - a)
        if cur_e is None or a > cur_e:
            if cur_e is not None:
                busy += cur_e - cur_s
            cur_s, cur_e = a, e
        else:
            cur_e = max(cur_e, e)
    if cur_e is not None:
        busy += cur_e - cur_s
    wall = t1 - t0
    lines = ["# rocprofv3 --kernel-trace: idle time between dispatches over the timed steps",
             "command: " + command, note, "",
             "steps: %d (dispatches of %s with grid %d)" % (steps, kernel, gmax),
             "wall_us: %.1f" % (wall / 1e3), "busy_us: %.1f" % (busy / 1e3),
             "idle_us: %.1f" % ((wall - busy) / 1e3),
             "idle_fraction: %.4f" % ((wall - busy) / wall),
             "wall_us_per_step: %.2f" % (wall / 1e3 / steps),
             "idle_us_per_step: %.2f" % ((wall - busy) / 1e3 / steps), "",
             "%-72s %7s %12s %12s" % ("kernel", "calls", "avg_us", "total_us")]
    for name, d in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        lines.append("%-72s %7d %12.2f %12.1f" % (name[:72], len(d), sum(d) / len(d) / 1e3, sum(d) / 1e3))
    with open(out_path, "w") as fo:
        fo.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def counters_summary(csvs, out_path, command, note):
    """Text summary of rocprofv3 --pmc passes (one CSV each) for the tracked FP64 D2Q37 kernels:
    the mean of every counter per dispatch, and the pipeline ratios the counters give.
    GRBM_GUI_ACTIVE reads the sum of the 8 XCDs' busy cycles, and the TA, TD and TCP counters
    the sum of their 256 per-CU instances, so a unit's busy fraction is its _sum over
    32 x GRBM_GUI_ACTIVE; the SQ wave-cycle counters give fractions of the waves' lifetime."""
    import csv
    acc = {}
    for path in csvs:
        with open(path) as f:
            for r in csv.DictReader(f):
                acc.setdefault(r["Kernel_Name"], {}).setdefault(r["Counter_Name"], []).append(
                    float(r["Counter_Value"]))
    lines = ["# rocprofv3 --pmc: pipeline counters per dispatch", "command: " + command, note, ""]
    for short, name in TRACKED.items():
        if name not in acc:
            continue
        m = {k: sum(v) / len(v) for k, v in acc[name].items()}
        n = min(len(v) for v in acc[name].values())
        lines.append("%s (%s), %d dispatches per pass" % (short, name, n))
        for k in sorted(m):
            lines.append("  %-36s %14.1f" % (k, m[k]))
        g = m.get("GRBM_GUI_ACTIVE")
        if g:
            for k, label in (("TA_TA_BUSY_sum", "TA busy"), ("TD_TD_BUSY_sum", "TD busy"),
                             ("TCP_PENDING_STALL_CYCLES_sum", "TCP stalled on pending misses"),
                             ("TD_TC_STALL_sum", "TD stalled on the cache")):
                if k in m:
                    lines.append("  ratio %-38s %.3f" % (label, m[k] / (32.0 * g)))
        wc = m.get("SQ_WAVE_CYCLES")
        if wc:
            for k, label in (("SQ_WAIT_INST_ANY", "waves waiting on a dependency"),
                             ("SQ_ACTIVE_INST_VALU", "waves issuing VALU")):
                if k in m:
                    lines.append("  ratio %-38s %.3f" % (label, m[k] / wc))
        if m.get("SQ_WAVES"):
            for k in ("SQ_INSTS_VMEM_RD", "SQ_INSTS_VALU"):
                if k in m:
                    lines.append("  per wave %-35s %.1f" % (k, m[k] / m["SQ_WAVES"]))
        if "TCC_HIT_sum" in m and "TCC_MISS_sum" in m:
            lines.append("  ratio %-38s %.3f" % ("L2 hit rate", m["TCC_HIT_sum"] /
                                                  max(m["TCC_HIT_sum"] + m["TCC_MISS_sum"], 1.0)))
        lines.append("")
    with open(out_path, "w") as fo:
        fo.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def request_summary(csv_path, out_path, command, note):
    """HBM read bytes per dispatch from the L2's read requests to memory by size (one --pmc pass
    of TCC_EA0_RDREQ_{32B,64B,128B}_sum and TCC_EA0_RDREQ_sum): 32 n32 + 64 n64 + 128 n128.  This
    resolves what FETCH_SIZE, scaled by a copy whose requests are all 128-byte, counts twice for a
    kernel whose partial-line reads go out as 64- or 32-byte requests."""
    acc = pmc_means_all(csv_path)
    lines = ["# rocprofv3 --pmc: HBM read requests by size per dispatch", "command: " + command, note,
             "", "%-72s %12s %12s %12s %12s %12s" % ("kernel", "n32", "n64", "n128", "n_total",
                                                      "read MB")]
    for name, m in sorted(acc.items(), key=lambda kv: -kv[1].get("TCC_EA0_RDREQ_sum", 0.0)):
        n32 = m.get("TCC_EA0_RDREQ_32B_sum", 0.0)
        n64 = m.get("TCC_EA0_RDREQ_64B_sum", 0.0)
        n128 = m.get("TCC_EA0_RDREQ_128B_sum", 0.0)
        mb = (32 * n32 + 64 * n64 + 128 * n128) / 1e6
        lines.append("%-72s %12.0f %12.0f %12.0f %12.0f %12.2f" % (
            name[:72], n32, n64, n128, m.get("TCC_EA0_RDREQ_sum", 0.0), mb))
    for short, name in TRACKED.items():
        if name in acc:
            m = acc[name]
            rd = 32 * m.get("TCC_EA0_RDREQ_32B_sum", 0.0) + 64 * m.get("TCC_EA0_RDREQ_64B_sum", 0.0) + \
                128 * m.get("TCC_EA0_RDREQ_128B_sum", 0.0)
            lines.append("read_bytes_by_request_%s: %d" % (short, round(rd)))
    with open(out_path, "w") as fo:
        fo.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def pmc_means_all(path):
    """Mean value per dispatch of every counter, per kernel name, from a rocprofv3 --pmc CSV."""
    import csv
    acc = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            acc.setdefault(row["Kernel_Name"], {}).setdefault(row["Counter_Name"], []).append(
                float(row["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in acc.items()}


def recorded_traffic(short):
    """HBM bytes per launch of a tracked kernel ("grid", "frame" or "bulk") from the committed
    counter summary, or None when it is missing or was taken from another version of the
    kernels."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as f:
            for ln in f:
                if ":" in ln:
                    k, v = ln.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_source_sha256") != kernel_source_hash():
            return None
        return int(kv["traffic_%s_bytes_per_launch" % short])
    except (OSError, KeyError, ValueError):
        return None


def host_cpu():
    """(model name, physical cores) of this host, from /proc/cpuinfo."""
    model, cores = None, set()
    try:
        phys = core = None
        with open("/proc/cpuinfo") as f:
            for ln in f:
                k, _, v = ln.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and model is None:
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
        if phys is not None:
            cores.add((phys, core))
    except OSError:
        pass
    return model, (len(cores) or None)


def roofline_entry(R, args, storage, copy_gbs):
    """The roofline object of the bench line: the dominant kernel of the timed steps (the grid
    of phase A and the bulk tiles in the fused schedule, else the bulk kernel), with the frame
    kernel and the whole step beside it."""
    fused = args.overlap == 2
    tracked = storage == "f64" and args.L == 1024 and args.W == 32 and args.bc == "nrbc" and \
        args.layout == 0 and args.bulk_tx == 64 and fused
    gbs, fgbs = R.get("grid_gbs"), R.get("frame_gbs")
    return {
        "bound": "hbm",
        "kernel": "k_phase_a_bulk (bulk stream-collide tiles, and phase A: the characteristic ring "
                  "fill and the PML auxiliary update, one grid)"
                  if fused else "k_bulk (interior stream-collide)",
        "achieved": round(gbs, 1) if gbs else None,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(gbs / HBM_PEAK_GBS, 4) if gbs else None,
        "traffic": recorded_traffic("grid" if fused else "bulk") if tracked else None,
        "bytes_per_launch": R["grid_bytes_per_launch"],
        "avg_launch_ms": round(R["grid_kernel_ms"], 5),
        "frame_kernel": {
            "kernel": "k_frame (collision of the boundary layers and the PML, with the PML term)",
            "achieved": round(fgbs, 1) if fgbs else None,
            "frac": round(fgbs / HBM_PEAK_GBS, 4) if fgbs else None,
            "traffic": recorded_traffic("frame") if tracked else None,
            "bytes_per_launch": R["frame_bytes_per_launch"],
            "avg_launch_ms": round(R["frame_kernel_ms"], 5),
        },
        "whole_step": {"achieved": round(R["gbs_step"], 1), "frac": round(R["frac_step"], 4),
                       "ms_per_step": round(R["ms_per_step"], 5)},
        "device_copy_gbs": round(copy_gbs, 1) if copy_gbs else None,
        "frac_of_device_copy": round(gbs / copy_gbs, 4) if copy_gbs and gbs else None,
        "timing": "HIP events attached to the dispatch of the step grid and of the frame kernel "
                  "(hipExtLaunchKernelGGL) on every fourth of the timed %d steps (%d launches each), "
                  "on the stream they run on" % (args.steps, R["launches_timed"]),
    }


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
    ap.add_argument("--overlap", type=int, default=2,
                    help="0: kernels in order; 1: boundary/PML chain on a side stream beside the "
                         "bulk kernel; 2: phase A fused with the bulk tiles in one grid")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=300)
    ap.add_argument("--prof-steps", type=int, default=500,
                    help="steps of a separate pass that runs the kernel classes in order and times "
                         "each (0 skips it)")
    ap.add_argument("--large-steps", type=int, default=200,
                    help="timed steps per run of the 4224^2 leg (0 skips it)")
    ap.add_argument("--large-bcs", default="zg,nrbc")
    ap.add_argument("--large-error-steps", type=int, default=2000,
                    help="4224^2 runs continue to this step count; FP32 and FP16 moments are then "
                         "compared with FP64 (0 skips)")
    ap.add_argument("--d2q9-steps", type=int, default=1000,
                    help="timed steps of the D2Q9 leg at the main size (0 skips it)")
    ap.add_argument("--d2q17-steps", type=int, default=1000,
                    help="timed steps of the D2Q17 leg at the main size (0 skips it)")
    ap.add_argument("--batch-runs", type=int, default=256, help="0 skips the batch sweep")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--serve-jobs", type=int, default=24, help="0 skips the serving trace")
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-scale", type=float, default=1.0,
                    help="multiplier on the trace's step counts (1000-20000)")
    ap.add_argument("--serve-tick", type=int, default=200, help="steps per serving tick")
    ap.add_argument("--serve-sustain-jobs", type=int, default=12,
                    help="arrivals of a second trace at a sustainable rate (0 skips it)")
    ap.add_argument("--serve-sustain-rate", type=float, default=1.0)
    ap.add_argument("--no-copy-bw", dest="copy_bw", action="store_false",
                    help="skip timing a plain 2 GiB device copy (attainable HBM bandwidth)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of 1 GiB (HBM counter calibration)")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "OUT"),
                    help="summarise two rocprofv3 --pmc passes into OUT and exit (no GPU)")
    ap.add_argument("--pmc-command", default="", help="command line recorded in the summary")
    ap.add_argument("--stats-summary", nargs=2, metavar=("STATS_CSV", "OUT"),
                    help="summarise a rocprofv3 --kernel-trace --stats CSV into OUT and exit (no GPU)")
    ap.add_argument("--stats-command", default="", help="command line recorded in the summary")
    ap.add_argument("--stats-note", default="", help="workload note recorded in the summary")
    ap.add_argument("--counters-summary", nargs="+", metavar="CSV",
                    help="pipeline-counter summary of --pmc CSVs (the last argument is the output "
                         "file) and exit")
    ap.add_argument("--request-summary", nargs=2, metavar=("PMC_CSV", "OUT"),
                    help="write HBM read bytes by request size from a --pmc pass and exit")
    ap.add_argument("--gaps-summary", nargs=2, metavar=("TRACE_CSV", "OUT"),
                    help="write the idle time between dispatches of a rocprofv3 kernel trace and exit")
    ap.add_argument("--gaps-steps", type=int, default=200, help="timed steps in the trace")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary, command=args.pmc_command)
        return
    if args.stats_summary:
        stats_summary(*args.stats_summary, command=args.stats_command, note=args.stats_note)
        return
    if args.request_summary:
        request_summary(*args.request_summary, command=args.stats_command, note=args.stats_note)
        return
    if args.counters_summary:
        counters_summary(args.counters_summary[:-1], args.counters_summary[-1],
                         command=args.stats_command, note=args.stats_note)
        return
    if args.gaps_summary:
        gaps_summary(*args.gaps_summary, command=args.stats_command, note=args.stats_note,
                     steps=args.gaps_steps)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU only (no multi-GPU path); use --gpus 1",
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
    spec = wl.vortex_pulse(L=args.L, W=args.W, sigma_max=args.sigma, mach=args.mach, bc=args.bc)
    for storage in args.storages.split(","):
        _log("bench: storage", storage)
        r = run_from_spec(lbm, spec, storage, stream, alloc, args.layout, args.bulk_tx, args.overlap)
        results[storage] = measure(torch, lbm, r, spec, storage, args.steps, args.warmup,
                                   args.prof_steps, args.overlap == 2)
        if storage != "f64" and "f64" in results:
            results[storage]["err_vs_f64"] = moment_errors(r.moments(), results["f64"]["_moments"])
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
        "roofline": roofline_entry(R, args, main_s, copy_gbs),
        "variants": {},
    }
    def rnd(v):
        # six significant digits: errors of 1e-9 must survive
        if isinstance(v, dict):
            return {k: rnd(x) for k, x in v.items() if not k.startswith("_")}
        return float("%.6g" % v) if isinstance(v, float) else v
    for s, v in results.items():
        line["variants"][s] = rnd(v)
    if args.large_steps > 0:
        line["at_4224"] = rnd(large_leg(torch, lbm, wl, args))
    if args.d2q17_steps > 0:
        line["d2q17"] = rnd(d2q17_leg(torch, lbm, wl, args))
    if args.d2q9_steps > 0:
        line["d2q9"] = rnd(d2q9_leg(torch, lbm, wl, args))
    if args.batch_runs > 0:
        _log("bench: batch sweep")
        line["batch"] = rnd(batch_leg(torch, lbm, wl, args))
    if args.serve_jobs > 0:
        _log("bench: serving trace")
        line["serving"] = {"arrivals": serve_trace(args.serve_jobs, args.serve_rate, args.serve_scale,
                                                   "f32", args.serve_tick)}
        if args.serve_sustain_jobs > 0:
            _log("bench: serving trace at a sustainable rate")
            line["serving"]["sustainable"] = serve_trace(args.serve_sustain_jobs, args.serve_sustain_rate,
                                                         args.serve_scale, "f32", args.serve_tick)
        if "batch" in line:
            line["serving"]["batch_group_mlups"] = line["batch"]["group_mlups"]
    if not args.no_cpu:
        _log("bench: cpu baseline (oracle)")
        mlups_cpu, threads, dt_cpu = cpu_baseline(wl, args.L, args.W, args.sigma, args.mach, args.bc,
                                                  args.cpu_steps)
        model, phys = host_cpu()
        line["cpu_baseline"] = {"value": round(mlups_cpu, 2), "unit": "MLUPS", "cores": threads,
                                "kind": "oracle",
                                "sample": "%d steps of the same %d^2 FP64 workload (%.1f s)"
                                          % (args.cpu_steps, args.L + 2 * args.W, dt_cpu),
                                "threads": threads, "physical_cores": phys, "cpu_model": model}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
