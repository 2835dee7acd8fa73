"""Scheduling logic of the serving loop on the CPU with a mock backend (no device)."""
import pytest

from paper_2504_20169_amd.serve import Engine, Job


class MockBackend:
    def __init__(self, bytes_per_node=100, fail_ids=()):
        self.bpn = bytes_per_node
        self.fail_ids = set(fail_ids)
        self.resident = {}
        self.launches = []
        self.log = []

    def footprint(self, job):
        return job.nodes * self.bpn

    def start(self, job):
        h = object()
        self.resident[id(h)] = [job, 0]
        self.log.append(("start", job.jid))
        return h

    def advance(self, handles, steps):
        self.launches.append(sorted(self.resident[id(h)][0].jid for h in handles))
        for h, s in zip(handles, steps):
            self.resident[id(h)][1] += s

    def sync(self):
        pass

    def healthy(self, h):
        job, done = self.resident[id(h)]
        return not (job.jid in self.fail_ids and done >= 2)

    def finish(self, h):
        job, done = self.resident.pop(id(h))
        self.log.append(("finish", job.jid))
        return {"steps": done}

    def drop(self, h):
        job, _ = self.resident.pop(id(h))
        self.log.append(("drop", job.jid))


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 0.001
        return self.t


def _job(k, L, steps, W=0):
    return Job(jid=k, L=L, W=W, steps=steps)


def test_budget_limits_resident_bytes_and_backfills():
    be = MockBackend()
    eng = Engine(be, hbm_budget=100 * (64 * 64 + 32 * 32), tick_steps=10, clock=Clock())
    big, big2, small = _job(0, 64, 30), _job(1, 64, 30), _job(2, 32, 10)
    for j in (big, big2, small):
        eng.submit(j)
    eng.tick()
    # big fits, big2 does not, the small job behind it is admitted (no head-of-line blocking)
    assert be.launches[0] == [0, 2]
    assert eng.used <= eng.budget
    while eng.active or eng.waiting:
        eng.tick()
        assert eng.used <= eng.budget
    assert all(j.status == "done" for j in eng.finished)
    assert {j.jid: j.result["steps"] for j in eng.finished} == {0: 30, 1: 30, 2: 10}


def test_continuous_batching_shares_launches():
    be = MockBackend()
    eng = Engine(be, hbm_budget=10 ** 12, tick_steps=5, clock=Clock())
    eng.submit(_job(0, 16, 20))
    eng.tick()
    eng.submit(_job(1, 16, 20))   # arrives while job 0 runs
    eng.tick()
    assert be.launches[0] == [0] and be.launches[1] == [0, 1]


def test_oversized_job_rejected_and_failed_job_isolated():
    be = MockBackend(fail_ids={1})
    eng = Engine(be, hbm_budget=100 * 40 * 40, tick_steps=1, clock=Clock())
    eng.submit(_job(9, 100, 5))        # larger than the whole budget
    eng.submit(_job(0, 16, 6))
    eng.submit(_job(1, 16, 6))
    while eng.active or eng.waiting:
        eng.tick()
    st = {j.jid: j.status for j in eng.finished}
    assert st == {9: "rejected", 0: "done", 1: "failed"}
    assert [j for j in eng.finished if j.jid == 0][0].result["steps"] == 6
    rep = eng.report()
    assert rep["done"] == 1 and rep["failed"] == 1 and rep["rejected"] == 1
    assert eng.used == 0


def test_trace_report_percentiles():
    be = MockBackend()
    eng = Engine(be, hbm_budget=10 ** 12, tick_steps=50, clock=Clock())
    jobs = [Job(jid=k, L=16, W=0, steps=100 + 10 * k, arrival=0.0) for k in range(20)]
    rep = eng.run_trace(jobs, realtime=False)
    assert rep["done"] == 20
    assert rep["p50_s"] <= rep["p99_s"]
    assert rep["aggregate_mlups"] > 0


class PreparingBackend(MockBackend):
    """Mock of a backend that builds admitted jobs off the tick path and checks the whole batch
    at once: a job's run is ready only after `delay` further polls."""

    def __init__(self, delay=2, fail_build=(), **kw):
        super().__init__(**kw)
        self.delay = delay
        self.fail_build = set(fail_build)
        self.checks = 0

    def prepare(self, job):
        be = self

        class Pending:
            polls = 0

            def done(self):
                self.polls += 1
                return self.polls > be.delay

            def result(self):
                if job.jid in be.fail_build:
                    raise RuntimeError("setup failed")
                return ("run", job.jid)

        return Pending()

    def start(self, job, run=None):
        assert run == ("run", job.jid)
        return super().start(job)

    def check_all(self, handles):
        self.checks += 1
        return [self.healthy(h) for h in handles]


def test_prepared_jobs_join_when_ready_and_failed_setup_is_retired():
    be = PreparingBackend(delay=2, fail_build=[3])
    eng = Engine(be, hbm_budget=10 ** 9, tick_steps=10, clock=Clock())
    for k in range(4):
        eng.submit(_job(k, 16, 30))
    eng.tick()                        # nothing resident yet: the engine waits for all prepared runs
    assert be.launches[0] == [0, 1, 2]
    eng.submit(_job(4, 16, 20))
    eng.tick()                        # job 4 is still being prepared: the others step without it
    assert be.launches[1] == [0, 1, 2]
    while eng.active or eng.waiting or eng.preparing:
        eng.tick()
    st = {j.jid: j.status for j in eng.finished}
    assert st == {0: "done", 1: "done", 2: "done", 3: "failed", 4: "done"}
    assert eng.used == 0
    assert be.checks == len(be.launches)   # one batch check per tick
