"""The serving scheduler on the CPU: admission by memory budget, continuous batching at tick
boundaries, latency accounting, rejection and cancellation. The executor here is a stand-in
that steps each job with the CPU oracle (restarts of the oracle are bitwise) on a virtual
clock that advances by a fixed cost per site-update."""
import numpy as np
import pytest

from paper_2603_22553_amd import serve, synth


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, d):
        self.t += max(d, 0.0)


class OracleExecutor:
    SECONDS_PER_SU = 1e-9
    BYTES_PER_SITE = 100

    def __init__(self, oracle, clock):
        self.o = oracle
        self.clock = clock
        self.step_calls = []

    def footprint(self, job):
        return job.n_sites * self.BYTES_PER_SITE

    def start(self, job):
        f = job.fields
        r = self.o.run(f.F, f.delta, f.region, f.n_regions, 0, moments=False)
        return {"state": (r.rho, r.re, r.im, None, None), "rec": [r.records], "job": job}

    def step(self, handles, steps):
        self.step_calls.append(list(steps))
        for h, s in zip(handles, steps):
            f = h["job"].fields
            r = self.o.run(f.F, f.delta, f.region, f.n_regions, s, state=h["state"])
            h["state"] = (r.rho, r.re, r.im, None, None)
            h["rec"].append(r.records[1:])
            self.clock.t += s * h["job"].n_sites * self.SECONDS_PER_SU

    def finish(self, job, h):
        rec = np.concatenate(h["rec"])
        R = job.fields.n_regions
        G = rec[:, 0:2 * R:2].sum(1) + 1j * rec[:, 1:2 * R:2].sum(1)
        return {"fid": G, "peak_ppm": self.o.peak_ppm(G, 5e-6, 400e6)}

    def cancel(self, h):
        pass


def trace(n, rate=50.0, seed=7, sides=(8, 14), steps=(150, 400)):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1 / rate, size=n))
    jobs = []
    for j in range(n):
        side = int(rng.integers(sides[0], sides[1] + 1))
        f = synth.particle(side, (side - 4) // 2, 1.5, (0.7, 2.0), seed=100 + j)
        jobs.append(serve.Job(j, float(t[j]), f, int(rng.integers(steps[0], steps[1] + 1))))
    return jobs


def solo_fid(oracle, job):
    f = job.fields
    return oracle.run(f.F, f.delta, f.region, f.n_regions, job.n_steps, moments=False).fid()


def test_every_job_matches_its_solo_run(oracle):
    clock = Clock()
    ex = OracleExecutor(oracle, clock)
    srv = serve.Server(ex, hbm_budget_bytes=1e12, tick_steps=100, clock=clock, sleep=clock.sleep)
    jobs = trace(12)
    st = srv.run(jobs)
    assert st["jobs_done"] == 12 and st["jobs_rejected"] == 0
    for j in jobs:
        assert j.status == "done"
        assert np.array_equal(j.result["fid"], solo_fid(oracle, j))
    # several jobs shared ticks (the batch held more than one lattice)
    assert max(len(c) for c in ex.step_calls) > 1


def test_budget_admission_and_queueing(oracle):
    clock = Clock()
    ex = OracleExecutor(oracle, clock)
    jobs = trace(10, rate=1e6)                      # all arrive at once
    budget = 2.5 * max(j.n_sites for j in jobs) * OracleExecutor.BYTES_PER_SITE
    srv = serve.Server(ex, hbm_budget_bytes=budget, tick_steps=80, clock=clock, sleep=clock.sleep)
    peak = []
    real_start = ex.start

    def start(job):
        h = real_start(job)
        peak.append(srv.used_bytes + job.footprint)
        return h

    ex.start = start
    st = srv.run(jobs)
    assert st["jobs_done"] == 10
    assert max(peak) <= budget and st["peak_resident_bytes"] <= budget
    # later jobs waited for memory: queueing time grows with arrival order
    q = [j.admitted_s - j.arrival_s for j in sorted(jobs, key=lambda j: j.job_id)]
    assert q[-1] > 0.0
    for j in jobs:
        assert j.latency_s == pytest.approx((j.admitted_s - j.arrival_s) + (j.finished_s - j.admitted_s))


def test_continuous_batching_joins_at_next_tick(oracle):
    """A job arriving while another runs is admitted at the next tick boundary."""
    clock = Clock()
    ex = OracleExecutor(oracle, clock)
    f = synth.particle(12, 4, 1.5, (0.7, 2.0), seed=1)
    long_job = serve.Job(0, 0.0, f, 1000)
    tick_cost = 100 * f.F.size * OracleExecutor.SECONDS_PER_SU
    late = serve.Job(1, 2.5 * tick_cost, f, 200)
    srv = serve.Server(ex, hbm_budget_bytes=1e12, tick_steps=100, clock=clock, sleep=clock.sleep)
    srv.run([long_job, late])
    assert late.admitted_s == pytest.approx(3 * tick_cost)
    assert late.finished_s < long_job.finished_s           # it overtook the long job
    assert ex.step_calls[3] == [100, 100]                    # both in the same batch


def test_rejection_and_cancellation(oracle):
    clock = Clock()
    ex = OracleExecutor(oracle, clock)
    jobs = trace(6, rate=1e6)
    for j in jobs:
        j.arrival_s = 0.0
    big = serve.Job(99, 0.0, synth.particle(40, 16, 2.0, (0.7, 2.0), seed=3), 10)
    budget = 2 * max(j.n_sites for j in jobs) * OracleExecutor.BYTES_PER_SITE
    srv = serve.Server(ex, hbm_budget_bytes=budget, tick_steps=50, clock=clock, sleep=clock.sleep)
    srv._t0 = clock()
    for j in jobs + [big]:
        srv.submit(j)
    assert big.status == "rejected"
    srv.cancel(jobs[-1].job_id)                    # still pending: dropped at once
    assert jobs[-1].status == "cancelled"
    srv.tick()                                     # admits what fits, runs one tick
    resident_id = srv.resident[0][0].job_id
    srv.cancel(resident_id)                        # resident: leaves at the next tick
    while srv.tick():
        pass
    st = srv.stats()
    assert st["jobs_cancelled"] == 2 and st["jobs_rejected"] == 1 and st["jobs_done"] == 4
    assert srv.used_bytes == 0


class AsyncOracleExecutor(OracleExecutor):
    """The oracle stand-in with the asynchronous interface of the GPU executor: a tick is
    queued by step_async and completed by wait; starts record whether a tick was in flight."""

    def __init__(self, oracle, clock):
        super().__init__(oracle, clock)
        self.inflight = False
        self.starts_during_tick = 0

    def start(self, job):
        if self.inflight:
            self.starts_during_tick += 1
        return super().start(job)

    def step_async(self, handles, steps):
        self.inflight = True
        return handles, steps

    def wait(self, token):
        self.step(*token)
        self.inflight = False


def test_overlapped_ticks_match_solo_runs(oracle):
    """With an asynchronous executor the server admits jobs while a tick is queued; every job
    still ends on its solo run's bits, and every tick advances all resident jobs by the same
    number of steps (one batch phase), never past the job nearest its end."""
    clock = Clock()
    ex = AsyncOracleExecutor(oracle, clock)
    srv = serve.Server(ex, hbm_budget_bytes=1e12, tick_steps=100, clock=clock, sleep=clock.sleep)
    assert srv.overlap
    jobs = trace(12)
    st = srv.run(jobs)
    assert st["jobs_done"] == 12
    for j in jobs:
        assert np.array_equal(j.result["fid"], solo_fid(oracle, j))
    assert ex.starts_during_tick > 0
    for call in ex.step_calls:
        assert len(set(call)) == 1 and call[0] <= 100
