"""Serving loop: simulation jobs admitted against an HBM budget, resident on the device and
advanced together by batched launches (continuous batching), with per-job latency.

Each tick the engine (1) admits waiting jobs in arrival order while they fit the HBM budget and
the slot limit (a job that does not fit yet does not block smaller ones behind it; a job larger
than the whole budget is rejected), (2) moves admitted jobs whose state is ready into the batch,
(3) advances every resident job by up to ``tick_steps`` steps in one batched call -- jobs admitted
this tick share the launches of jobs already running -- and (4) checks every resident job's state
at once and retires finished jobs: moments are exported, device memory is released and the
latency (arrival to result) is recorded.  A job whose state fails the stability check is retired
with an error and does not disturb the others.

A backend that offers ``prepare`` builds an admitted job's run (its initial fields on the host and
their upload) on worker threads, off the tick path, so arrivals do not stall the batch; one that
offers ``check_all`` checks the whole batch with one synchronisation.  ``GpuBackend`` drives the
HIP library through ``lbm.Group`` and offers both; the CPU tests use mock backends.
"""
from __future__ import annotations

import time
from collections import deque
from concurrent.futures import Future, ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Any, Optional

import numpy as np


@dataclass
class Job:
    jid: int
    L: int
    W: int
    steps: int
    bc: str = "zg"
    seed: int = 0
    sigma_max: float = 0.0015
    mach: float = 0.1
    arrival: float = 0.0
    # filled by the engine
    admitted: Optional[float] = None
    finished: Optional[float] = None
    done_steps: int = 0
    status: str = "queued"          # queued | preparing | running | done | failed | rejected
    result: Any = None
    handle: Any = field(default=None, repr=False)
    pending: Any = field(default=None, repr=False)
    nbytes: int = 0

    @property
    def nodes(self):
        return (self.L + 2 * self.W) ** 2

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


class GpuBackend:
    """Runs jobs on the HIP library: one lbm.Run per job, all resident runs in one lbm.Group.
    Admitted jobs are built on `workers` threads (fields and upload on the run's own stream) and
    join the group once ready."""

    def __init__(self, storage="f32", stream=None, allocator=None, workers=4):
        from paper_2504_20169_amd import lbm
        self.lbm = lbm
        self.storage = storage
        self.stream = stream
        self.allocator = allocator
        self.group = lbm.Group(stream=stream, allocator=allocator)
        self.pool = ThreadPoolExecutor(max_workers=workers) if workers > 0 else None

    def _make(self, job: Job):
        lbm = self.lbm
        r = lbm.Run(job.L, job.L, 0.8, 1.0, job.mach, 0.0, 1.0, storage=self.storage,
                    allocator=self.allocator)
        r.set_bc(lbm.LBM_ALL, job.bc)
        if job.W > 0:
            r.set_pml(lbm.LBM_ALL, job.W, job.sigma_max)
        return r

    def footprint(self, job: Job) -> int:
        r = self._make(job)
        b = r.footprint()
        r.close()
        return b

    def _build(self, job: Job):
        from paper_2504_20169_amd import workloads as wl
        r = self._make(job)
        spec = wl.vortex_pulse(L=job.L, W=job.W, sigma_max=job.sigma_max, mach=job.mach,
                               bc=job.bc, seed=job.seed, radius=min(16.0, job.L / 8.0))
        r.init(*spec.fields.as_tuple())
        return r

    def prepare(self, job: Job):
        """A future of the job's initialised run, built off the caller's thread (on the caller's
        thread when the backend has no workers)."""
        if self.pool is None:
            fut = Future()
            try:
                fut.set_result(self._build(job))
            except Exception as exc:        # reported when the engine joins the job
                fut.set_exception(exc)
            return fut
        return self.pool.submit(self._build, job)

    def start(self, job: Job, run=None):
        r = run if run is not None else self._build(job)
        self.group.add(r)
        return r

    def advance(self, handles, steps):
        if handles:
            order = {id(r): k for k, r in enumerate(self.group.members)}
            arr = np.zeros(len(self.group.members), dtype=np.int64)
            for r, s in zip(handles, steps):
                arr[order[id(r)]] = s
            self.group.step(steps=arr)

    def sync(self):
        self.group.synchronize()

    def healthy(self, r) -> bool:
        return r.check() == self.lbm.LBM_OK

    def check_all(self, handles):
        """Health of each handle, from one check of the whole group."""
        flags = self.group.check()
        order = {id(r): k for k, r in enumerate(self.group.members)}
        return [flags[order[id(r)]] == 0 for r in handles]

    def finish(self, r):
        rho, ux, uy, T = r.moments()
        self.group.remove(r)
        r.close()
        return dict(rho=rho, ux=ux, uy=uy, T=T)

    def drop(self, r):
        self.group.remove(r)
        r.close()

    def discard(self, run):
        """Release a prepared run that never joined the group."""
        run.close()

    def close(self):
        if self.pool is not None:
            self.pool.shutdown(wait=True)
        self.group.close()


class Engine:
    def __init__(self, backend, hbm_budget: int, max_jobs: int = 1024, tick_steps: int = 200,
                 clock=time.perf_counter):
        self.backend = backend
        self.budget = int(hbm_budget)
        self.max_jobs = max_jobs
        self.tick_steps = tick_steps
        self.clock = clock
        self.waiting: deque[Job] = deque()
        self.preparing: list[Job] = []
        self.active: list[Job] = []
        self.finished: list[Job] = []
        self.used = 0
        self.node_updates = 0
        self.t0 = None

    def submit(self, job: Job):
        job.nbytes = self.backend.footprint(job)
        if job.nbytes > self.budget:
            job.status = "rejected"
            job.finished = self.clock()
            self.finished.append(job)
            return
        self.waiting.append(job)

    def _admit(self, now):
        keep = deque()
        prep = getattr(self.backend, "prepare", None)
        while self.waiting:
            job = self.waiting.popleft()
            if len(self.active) + len(self.preparing) < self.max_jobs and \
                    self.used + job.nbytes <= self.budget:
                job.admitted = now
                self.used += job.nbytes
                if prep is not None:
                    job.pending = prep(job)
                    job.status = "preparing"
                    self.preparing.append(job)
                else:
                    job.handle = self.backend.start(job)
                    job.status = "running"
                    self.active.append(job)
            else:
                keep.append(job)
        self.waiting = keep

    def _join_ready(self, wait):
        """Move prepared jobs into the batch (all of them if `wait`, else the ready ones)."""
        still = []
        for j in self.preparing:
            if wait or j.pending.done():
                try:
                    run = j.pending.result()
                except Exception as exc:          # the job could not be set up: retire it
                    j.pending = None
                    j.status = "failed"
                    j.result = dict(error=str(exc))
                    j.finished = self.clock()
                    self.used -= j.nbytes
                    self.finished.append(j)
                    continue
                j.handle = self.backend.start(j, run)
                j.pending = None
                j.status = "running"
                self.active.append(j)
            else:
                still.append(j)
        self.preparing = still

    def tick(self):
        now = self.clock()
        if self.t0 is None:
            self.t0 = now
        self._admit(now)
        # with nothing resident, wait for the jobs being prepared instead of spinning
        self._join_ready(wait=not self.active)
        if not self.active:
            return 0
        steps = [min(self.tick_steps, j.steps - j.done_steps) for j in self.active]
        self.backend.advance([j.handle for j in self.active], steps)
        self.backend.sync()
        for j, s in zip(self.active, steps):
            j.done_steps += s
            self.node_updates += j.nodes * s
        check_all = getattr(self.backend, "check_all", None)
        if check_all is not None:
            ok = check_all([j.handle for j in self.active])
        else:
            ok = [self.backend.healthy(j.handle) for j in self.active]
        still = []
        for j, good in zip(self.active, ok):
            if not good:
                self.backend.drop(j.handle)
                j.status = "failed"
            elif j.done_steps >= j.steps:
                j.result = self.backend.finish(j.handle)
                j.status = "done"
            else:
                still.append(j)
                continue
            j.finished = self.clock()
            j.handle = None
            self.used -= j.nbytes
            self.finished.append(j)
        self.active = still
        return len(steps)

    def run_trace(self, jobs, realtime=True, log=None):
        """Feed jobs at their arrival times (seconds from start) and run until all finish."""
        pending = deque(sorted(jobs, key=lambda j: j.arrival))
        start = self.clock()
        for j in pending:
            j.arrival = start + j.arrival
        while pending or self.waiting or self.active or self.preparing:
            now = self.clock()
            while pending and (pending[0].arrival <= now or not realtime):
                self.submit(pending.popleft())
            if not self.active and not self.waiting and not self.preparing:
                if pending and realtime:
                    time.sleep(max(0.0, min(0.05, pending[0].arrival - self.clock())))
                continue
            n = self.tick()
            if log:
                log("tick: %d active, %d waiting, %d done, used %.2f GB" % (
                    n, len(self.waiting), len(self.finished), self.used / 1e9))
        self.elapsed = self.clock() - start
        return self.report()

    def report(self):
        done = [j for j in self.finished if j.status == "done"]
        lat = np.array([j.latency for j in done]) if done else np.zeros(0)
        el = getattr(self, "elapsed", None) or ((self.clock() - self.t0) if self.t0 else 0.0)
        return dict(
            jobs=len(self.finished), done=len(done),
            failed=sum(j.status == "failed" for j in self.finished),
            rejected=sum(j.status == "rejected" for j in self.finished),
            p50_s=float(np.percentile(lat, 50)) if len(lat) else None,
            p99_s=float(np.percentile(lat, 99)) if len(lat) else None,
            mean_s=float(lat.mean()) if len(lat) else None,
            elapsed_s=el,
            aggregate_mlups=self.node_updates / el / 1e6 if el > 0 else None,
        )


def jobs_from_trace(trace, scale_steps=1.0, sigma_max=0.0015):
    """Jobs from workloads.poisson_trace entries (arrival offset, dict)."""
    out = []
    for k, (t, d) in enumerate(trace):
        out.append(Job(jid=k, L=d["L"], W=d["W"], steps=max(1, int(d["steps"] * scale_steps)),
                       bc=d["bc"], seed=d["seed"], arrival=t, sigma_max=sigma_max))
    return out


def main():
    import argparse
    import json
    import sys

    from paper_2504_20169_amd import workloads as wl

    ap = argparse.ArgumentParser(description="serve a Poisson trace of D2Q37 jobs")
    ap.add_argument("--jobs", type=int, default=40)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--tick-steps", type=int, default=200)
    ap.add_argument("--scale-steps", type=float, default=1.0)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--seed", type=int, default=5)
    args = ap.parse_args()
    trace = wl.poisson_trace(args.jobs, rate=args.rate, seed=args.seed)
    jobs = jobs_from_trace(trace, args.scale_steps)
    be = GpuBackend(storage=args.storage)
    eng = Engine(be, int(args.budget_gb * 1e9), tick_steps=args.tick_steps)
    rep = eng.run_trace(jobs, log=lambda m: print(m, file=sys.stderr, flush=True))
    rep.update(rate=args.rate, budget_gb=args.budget_gb, storage=args.storage,
               scale_steps=args.scale_steps)
    print(json.dumps(rep))
    be.close()


if __name__ == "__main__":
    main()
