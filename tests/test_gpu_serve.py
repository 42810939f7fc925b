"""Continuous-batching server on the GPU: results in the mix equal results alone, bit for bit,
and a sampled job agrees with the CPU oracle."""
import numpy as np
import pytest

from conftest import rel_l2
from paper_2603_22553_amd import serve, synth

pytestmark = pytest.mark.gpu


def small_trace(n=8, seed=11):
    rng = np.random.default_rng(seed)
    jobs = []
    t = 0.0
    for j in range(n):
        t += float(rng.exponential(0.01))
        side = int(rng.integers(16, 33))
        f = synth.particle(side, (side - 8) // 2, 3.0, (0.7, 2.0), seed=500 + j)
        jobs.append(serve.Job(j, t, f, int(rng.integers(300, 1500))))
    return jobs


def test_served_equals_alone_and_oracle(oracle):
    from paper_2603_22553_amd.lattice import Lattice
    jobs = small_trace()
    srv = serve.Server(serve.GpuExecutor(), hbm_budget_bytes=200e9, tick_steps=200)
    st = srv.run(jobs)
    assert st["jobs_done"] == len(jobs)
    assert st["latency_p99_s"] >= st["latency_p50_s"] > 0
    for j in jobs:
        f = j.fields
        nz, ny, nx = f.F.shape
        with Lattice((nx, ny, nz), precision="mixed", track=("fid",), n_regions=f.n_regions,
                     max_records=j.n_steps + 1, batched=True) as lat:
            lat.set_fields(f)
            lat.init_state("uniform")
            lat.run(j.n_steps)
            assert np.array_equal(j.result["fid"], lat.fid())
            assert j.result["peak_ppm"] == lat.peak_ppm()
    j = jobs[3]
    o = oracle.run(j.fields.F, j.fields.delta, j.fields.region, j.fields.n_regions, j.n_steps,
                   moments=False)
    assert rel_l2(j.result["fid"], o.fid()) <= 1e-3
    assert abs(j.result["peak_ppm"] - oracle.peak_ppm(o.fid(), 5e-6, 400e6)) <= 0.01


def test_budget_queues_on_gpu():
    jobs = small_trace(6, seed=12)
    ex = serve.GpuExecutor()
    budget = 1.5 * max(ex.footprint(j) for j in jobs)
    srv = serve.Server(ex, hbm_budget_bytes=budget, tick_steps=300)
    st = srv.run(jobs)
    assert st["jobs_done"] == 6 and st["peak_resident_bytes"] <= budget
