"""Long parity runs of the GPU path against the oracle at the benchmark configurations' full
sizes. They take minutes of host time each, so pytest does not collect them; run them
directly on a GPU machine:

    python -u tests/long_validation.py particle   # 256^3 particle, first 2000 steps, FP64 + mixed
    python -u tests/long_validation.py particle_inputs   # mixed against the oracle on FP32 fields
    python -u tests/long_validation.py serve      # the sampled served job, its full length
    python -u tests/long_validation.py batch      # 8 of the 512 batched particles, 20 000 steps
    python -u tests/long_validation.py film       # 2048 x 256 x 256 film, first 200 steps

The oracle runs in segments (continuing from its own state), with a line printed after each,
and every case ends with one JSON line: FID relative L2 over all samples, the largest
relative uptake and moment errors, the spectral peaks and the total-population drift.
Tolerances: FID relative L2 <= 1e-5 (FP64) and <= 1e-3 (mixed), peaks within 0.01 ppm,
mass conserved to 1e-12.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

from oracle import oracle  # noqa: E402
from paper_2603_22553_amd import synth  # noqa: E402

DT, NU0 = 5e-6, 400e6


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def oracle_segments(f, steps, seg, bc=(0, 0, 0), init="uniform", moments=True):
    """Records of an oracle run of `steps` steps, taken in segments of `seg` steps."""
    rows, state, done = [], None, 0
    while done < steps:
        n = min(seg, steps - done)
        t = time.perf_counter()
        res = oracle.run(f.F, f.delta, f.region, f.n_regions, n, bc=bc, init=init,
                         moments=moments, state=state)
        rows.append(res.records if not rows else res.records[1:])
        state = (res.rho, res.re, res.im, res.M1, res.M2)
        done += n
        log(f"  oracle {done}/{steps} steps ({time.perf_counter() - t:.1f} s)")
    return np.concatenate(rows), state


def compare(tag, rec, ref, R, dt=DT, nu0=NU0):
    G = rec[:, 0:2 * R:2].sum(1) + 1j * rec[:, 1:2 * R:2].sum(1)
    Gr = ref[:, 0:2 * R:2].sum(1) + 1j * ref[:, 1:2 * R:2].sum(1)
    U, Ur = rec[:, 2 * R:3 * R], ref[:, 2 * R:3 * R]
    mass = U.sum(1)
    out = {"case": tag, "samples": int(G.size),
           "fid_rel_l2": float(np.linalg.norm(G - Gr) / np.linalg.norm(Gr)),
           "uptake_max_rel": float(np.max(np.abs(U - Ur)) / np.max(np.abs(Ur))),
           "mass_drift": float(np.max(np.abs(mass / mass[0] - 1.0))),
           "peak_ppm": float(oracle.peak_ppm(G, dt, nu0)),
           "peak_ppm_oracle": float(oracle.peak_ppm(Gr, dt, nu0))}
    if rec.shape[1] > 3 * R:
        S2, S2r = rec[:, 3 * R + 3:], ref[:, 3 * R + 3:]
        out["msd_max_rel"] = float(np.max(np.abs(S2 - S2r)) / max(np.max(np.abs(S2r)), 1e-300))
    return out


def gpu_records(f, steps, precision, bc=("periodic",) * 3, init="uniform", track=("fid", "msd"),
                chunk=5000):
    from paper_2603_22553_amd.lattice import Lattice
    with Lattice(f.shape_xyz, bc=bc, precision=precision, track=track, n_regions=f.n_regions,
                 max_records=steps + 1) as lat:
        lat.set_fields(f)
        lat.init_state(init)
        done = 0
        while done < steps:
            n = min(chunk, steps - done)
            lat.run(n)
            lat.synchronize()
            done += n
        log(f"  gpu {precision} {steps} steps done")
        return lat.records()


def case_particle(steps=2000):
    f = synth.single_particle_large()
    log(f"256^3 particle, {steps} steps")
    gpu = {p: gpu_records(f, steps, p) for p in ("fp64", "mixed")}
    ref, _ = oracle_segments(f, steps, 100)
    for p, rec in gpu.items():
        print(json.dumps(compare(f"particle 256^3 {p} {steps} steps", rec, ref, 2)), flush=True)


def case_particle_inputs(steps=2000):
    """The mixed path's error split in two: against the oracle on its own FP64 fields, and
    against the oracle on the fields rounded to FP32 as the mixed path stores them (what
    remains is the arithmetic of the mixed path)."""
    f = synth.single_particle_large()
    g = synth.Fields(f.F.astype(np.float32).astype(np.float64),
                     f.delta.astype(np.float32).astype(np.float64), f.region, f.n_regions)
    log(f"256^3 particle, {steps} steps, oracle on FP32-rounded fields")
    rec = gpu_records(f, steps, "mixed")
    ref, _ = oracle_segments(g, steps, 100)
    print(json.dumps(compare(f"particle 256^3 mixed vs oracle on FP32-rounded fields, {steps} steps",
                             rec, ref, 2)), flush=True)


def case_serve(n_requests=100):
    trace = synth.serving_trace(n_requests, rate_hz=20.0)
    j = trace[0]                                   # the every-100th sample of the trace
    f = synth.request_fields(j)
    log(f"served job {j.job_id}: {f.shape_xyz}, {j.n_steps} steps, mixed FID only")
    rec = gpu_records(f, j.n_steps, "mixed", track=("fid",))
    ref, _ = oracle_segments(f, j.n_steps, 2500, moments=False)
    print(json.dumps(compare(f"served job {j.job_id} {f.shape_xyz} {j.n_steps} steps", rec,
                             ref, f.n_regions)), flush=True)


def case_batch(steps=20000, sample=8):
    from paper_2603_22553_amd.lattice import Batch, Lattice
    specs = synth.batch_specs(512, 2000)
    radii = np.array([s.radius for s in specs])
    rng = np.random.default_rng(7)
    pick = [int(np.argmin(radii)), int(np.argmax(radii))]
    pick += [int(v) for v in rng.choice([k for k in range(512) if k not in pick], sample - 2,
                                        replace=False)]
    log(f"512 batched particles, {steps} steps; oracle on {pick}")
    fields = [synth.batch_particle(s) for s in specs]
    lats = []
    for f in fields:
        lat = Lattice(f.shape_xyz, precision="mixed", n_regions=f.n_regions, max_records=steps + 1,
                      batched=True)
        lat.set_fields(f)
        lat.init_state("uniform")
        lats.append(lat)
    b = Batch(lats)
    for k in range(0, steps, 2000):
        b.run(min(2000, steps - k))
        b.stream.synchronize()
        log(f"  batch {k + 2000}/{steps} steps")
    b.close()
    recs = {k: lats[k].records() for k in pick}
    for lat in lats:
        lat.close()
    for k in pick:
        f = fields[k]
        log(f"particle {k}: R {specs[k].radius}, {f.shape_xyz}")
        ref, _ = oracle_segments(f, steps, 2000)
        print(json.dumps(compare(f"batch particle {k} (R {specs[k].radius}) mixed {steps} steps",
                                 recs[k], ref, f.n_regions)), flush=True)


def case_film(steps=200):
    f = synth.film()
    bc_o = (1, 0, 0)
    log(f"film {f.shape_xyz}, {steps} steps, mixed, Boltzmann start")
    rec = gpu_records(f, steps, "mixed", bc=("closed", "periodic", "periodic"), init="boltzmann")
    ref, _ = oracle_segments(f, steps, 10, bc=bc_o, init="boltzmann")
    print(json.dumps(compare(f"film 2048x256x256 mixed {steps} steps", rec, ref, 3)), flush=True)


if __name__ == "__main__":
    oracle.build(force=False)
    cases = {"particle": case_particle, "particle_inputs": case_particle_inputs,
             "serve": case_serve, "batch": case_batch, "film": case_film}
    for name in sys.argv[1:] or ["particle"]:
        cases[name]()
