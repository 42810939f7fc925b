"""Continuous-batching spectrum server over the batched lattice sweep.

Spectrum / adsorption jobs (one carbon particle each) arrive over time. The server keeps
the lattices of admitted jobs resident on the GPU, admits new jobs whenever the device
memory budget allows, and advances all resident jobs together with one batched sweep
(lpc_batch_run) per tick: jobs that arrive while others run join at the next tick, and
finished jobs leave at the end of the tick in which their last step ran. A tick advances
every resident job by the same number of steps, at most `tick_steps` and at most what the
job closest to its end still needs, so that each tick is one phase of the batch (one table
upload, launches replayed from one captured graph) and a finished job frees its memory at
once. Each job's result is bit for bit the one it gets when run alone, because the batched
sweep keeps every lattice's own tiles and reduction order.

With an executor that steps asynchronously (GpuExecutor), admission overlaps the sweep: the
server queues a tick, then, while the device runs it, starts the jobs that have arrived (field
uploads and start on a second stream; they join at the next tick), and only then waits for
the tick and reads the results of the jobs it finished.

The executor is pluggable: GpuExecutor drives liblpc; tests drive the scheduler with a
CPU stand-in and a virtual clock.
"""
from __future__ import annotations

import dataclasses
import math
import time
from collections import deque
from typing import Callable, List, Optional

import numpy as np


@dataclasses.dataclass
class Job:
    job_id: int
    arrival_s: float
    fields: object            # synth.Fields-like: F, delta, region (shape (nz, ny, nx)), n_regions
    n_steps: int
    bc: tuple = ("periodic", "periodic", "periodic")
    # filled in by the server
    admitted_s: Optional[float] = None
    finished_s: Optional[float] = None
    steps_done: int = 0
    result: Optional[dict] = None
    status: str = "pending"   # pending | resident | done | rejected | cancelled
    footprint: int = 0

    @property
    def n_sites(self) -> int:
        return int(np.prod(self.fields.F.shape))

    @property
    def latency_s(self) -> Optional[float]:
        return None if self.finished_s is None else self.finished_s - self.arrival_s


class GpuExecutor:
    """Runs jobs on one GPU through liblpc: float storage with double sums, FID only.

    The batched sweep runs on the device's current stream; each job's lattice (its field
    uploads, start and post-processing) lives on a second stream of the same priority, so
    that those overlap the sweep of the jobs already running. lpc_batch_run waits for the
    lattices' own streams before it steps them. With `tune`, each box configuration's plan
    comes from the autotuner (timed once per configuration, in a batch of copies)."""

    def __init__(self, precision: str = "mixed", track=("fid",), device: str = "cuda",
                 keep_fid: bool = True, tune: bool = False):
        import torch
        from . import lattice as _lat  # loads liblpc; fails loudly if it is not built
        self._lat = _lat
        self._torch = torch
        self.precision = precision
        self.track = tuple(track)
        self.device = device
        self.keep_fid = keep_fid
        self.tune = tune
        self.side = torch.cuda.Stream(device=device)          # default priority
        self.main = torch.cuda.current_stream(device)

    def _cfg(self, job: Job):
        nz, ny, nx = job.fields.F.shape
        return self._lat.make_config((nx, ny, nz), job.bc, self.precision, self.track,
                                     job.fields.n_regions, max_records=job.n_steps + 1,
                                     batched=True)

    def footprint(self, job: Job) -> int:
        return self._lat.footprint(self._cfg(job)) + self._lat.batch_footprint(1)

    def start(self, job: Job):
        nz, ny, nx = job.fields.F.shape
        lat = self._lat.Lattice((nx, ny, nz), job.bc, self.precision, self.track,
                                job.fields.n_regions, max_records=job.n_steps + 1,
                                device=self.device, batched=True, stream=self.side)
        if self.tune:
            from . import autotune
            autotune.apply(lat)
        lat.set_fields(job.fields)
        lat.init_state("uniform")
        return lat

    def step_async(self, handles: list, steps: List[int]):
        """Queues one tick on the main stream and returns at once (the batch waits for the
        lattices' own streams first); wait() blocks until it has run."""
        b = self._lat.Batch(handles, stream=self.main)
        b.run(steps)
        done = self._torch.cuda.Event()
        done.record(self.main)
        return b, done

    def wait(self, token) -> None:
        b, done = token
        done.synchronize()
        b.close()

    def step(self, handles: list, steps: List[int]) -> None:
        self.wait(self.step_async(handles, steps))

    def finish(self, job: Job, handle) -> dict:
        out = {"peak_ppm": handle.peak_ppm()}
        if self.keep_fid:
            out["fid"] = handle.fid()
        out["mass"] = handle.moments()[0][-1]
        handle.close()
        return out

    def cancel(self, handle) -> None:
        handle.close()


class Server:
    """Admission by memory budget, tick-based continuous batching, latency accounting."""

    def __init__(self, executor, hbm_budget_bytes: float = 200e9, tick_steps: int = 2000,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep, uniform_ticks: bool = True):
        self.ex = executor
        self.budget = float(hbm_budget_bytes)
        self.tick_steps = int(tick_steps)
        self.clock = clock
        self.sleep = sleep
        self.pending: deque = deque()
        self.resident: list = []        # (job, handle)
        self.done: list = []
        self.rejected: list = []
        self.cancelled: list = []
        self.used_bytes = 0
        self.peak_bytes = 0
        self.ticks = 0
        self.site_updates = 0
        self._t0 = None
        self._cancel_ids = set()
        self.uniform_ticks = uniform_ticks
        self.overlap = hasattr(executor, "step_async")
        self._to_retire: list = []       # finished in the last tick, results not yet read

    # ----------------------------------------------------------------- requests
    def now(self) -> float:
        return self.clock() - self._t0

    def submit(self, job: Job) -> None:
        job.footprint = int(self.ex.footprint(job))
        if job.footprint > self.budget:
            job.status = "rejected"
            self.rejected.append(job)
            return
        self.pending.append(job)

    def cancel(self, job_id: int) -> None:
        """Drops a pending job at once; a resident job leaves at the next tick boundary."""
        for j in list(self.pending):
            if j.job_id == job_id:
                self.pending.remove(j)
                j.status = "cancelled"
                self.cancelled.append(j)
                return
        self._cancel_ids.add(job_id)

    # ----------------------------------------------------------------- loop
    def _admit(self) -> None:
        now = self.now()
        while self.pending and self.pending[0].arrival_s <= now:
            job = self.pending[0]
            if self.used_bytes + job.footprint > self.budget:
                break                     # first come, first served: wait for memory
            self.pending.popleft()
            handle = self.ex.start(job)
            job.admitted_s = self.now()
            job.status = "resident"
            self.used_bytes += job.footprint
            self.peak_bytes = max(self.peak_bytes, self.used_bytes)
            self.resident.append((job, handle))

    def _retire(self, job: Job, handle, cancelled: bool = False) -> None:
        self.used_bytes -= job.footprint
        if cancelled:
            self.ex.cancel(handle)
            job.status = "cancelled"
            self.cancelled.append(job)
            return
        job.result = self.ex.finish(job, handle)
        job.finished_s = self.now()
        job.status = "done"
        self.done.append(job)

    def _tick_steps(self) -> List[int]:
        left = [j.n_steps - j.steps_done for j, _ in self.resident]
        if self.uniform_ticks:
            s = min(self.tick_steps, min(left))
            return [s] * len(left)
        return [min(self.tick_steps, n) for n in left]

    def _account(self, steps) -> None:
        keep = []
        for (job, h), s in zip(self.resident, steps):
            job.steps_done += s
            self.site_updates += s * job.n_sites
            if job.steps_done >= job.n_steps:
                self._to_retire.append((job, h))
            else:
                keep.append((job, h))
        self.resident = keep

    def _drain_retired(self) -> None:
        for job, h in self._to_retire:
            self._retire(job, h)
        self._to_retire = []

    def tick(self) -> bool:
        """Admits what fits, advances every resident job; False when nothing is left."""
        if self.overlap:
            return self._tick_overlapped()
        self._admit()
        if self._cancel_ids:
            keep = []
            for job, h in self.resident:
                if job.job_id in self._cancel_ids:
                    self._retire(job, h, cancelled=True)
                else:
                    keep.append((job, h))
            self.resident = keep
            self._cancel_ids.clear()
        if not self.resident:
            if not self.pending:
                return False
            wait = self.pending[0].arrival_s - self.now()
            if wait > 0:
                self.sleep(wait)
            return True
        steps = self._tick_steps()
        self.ex.step([h for _, h in self.resident], steps)
        self.ticks += 1
        self._account(steps)
        self._drain_retired()
        return True

    def _tick_overlapped(self) -> bool:
        """One tick with the admission work beside it: queue the tick, start the jobs that
        join at the next tick (their uploads run on the second stream while the device sweeps),
        wait, then read the results of the jobs that finished."""
        self._apply_cancels()
        if not self.resident:
            self._admit()
            if not self.resident:
                if not self.pending:
                    return False
                wait = self.pending[0].arrival_s - self.now()
                if wait > 0:
                    self.sleep(wait)
                return True
        steps = self._tick_steps()
        token = self.ex.step_async([h for _, h in self.resident], steps)
        self.ticks += 1
        running = self.resident
        self.resident = []
        self._admit()                      # uploads of jobs that join at the next tick
        admitted = self.resident
        self.resident = running
        self.ex.wait(token)
        self._account(steps)
        self._drain_retired()
        self.resident.extend(admitted)
        return True

    def _apply_cancels(self) -> None:
        if not self._cancel_ids:
            return
        keep = []
        for job, h in self.resident:
            if job.job_id in self._cancel_ids:
                self._retire(job, h, cancelled=True)
            else:
                keep.append((job, h))
        self.resident = keep
        self._cancel_ids.clear()

    def run(self, jobs: List[Job], progress: Optional[Callable[[dict], None]] = None,
            progress_every_s: float = 30.0) -> dict:
        """Serves a trace (jobs sorted by arrival) to completion and returns statistics;
        `progress` (optional) receives a short status dict every progress_every_s seconds."""
        self._t0 = self.clock()
        for j in sorted(jobs, key=lambda j: j.arrival_s):
            self.submit(j)
        last = self.now()
        while self.tick():
            if progress is not None and self.now() - last >= progress_every_s:
                last = self.now()
                progress({"t_s": last, "done": len(self.done), "resident": len(self.resident),
                          "pending": len(self.pending), "ticks": self.ticks})
        return self.stats()

    def stats(self) -> dict:
        lat = np.array([j.latency_s for j in self.done]) if self.done else np.zeros(0)
        queue = np.array([j.admitted_s - j.arrival_s for j in self.done]) if self.done else np.zeros(0)
        service = np.array([j.finished_s - j.admitted_s for j in self.done]) if self.done else np.zeros(0)
        span = max((j.finished_s for j in self.done), default=0.0)

        def pct(a, q):
            return float(np.percentile(a, q)) if a.size else math.nan

        return {
            "jobs_done": len(self.done),
            "jobs_rejected": len(self.rejected),
            "jobs_cancelled": len(self.cancelled),
            "makespan_s": span,
            "spectra_per_s": len(self.done) / span if span > 0 else math.nan,
            "latency_p50_s": pct(lat, 50), "latency_p99_s": pct(lat, 99),
            "queue_p50_s": pct(queue, 50), "queue_p99_s": pct(queue, 99),
            "service_p50_s": pct(service, 50), "service_p99_s": pct(service, 99),
            "site_updates_per_s": self.site_updates / span if span > 0 else math.nan,
            "ticks": self.ticks,
            "peak_resident_bytes": self.peak_bytes,
        }
