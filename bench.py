"""Benchmark of the lattice sweep on one MI355X.

Default workload (the headline line, `--workload film`): the supercapacitor film, a
2048 x 256 x 256 lattice (134 M sites) closed in x and periodic in y and z, with two
768-site porous electrodes (lognormal pore widths, median 0.9 and 1.3 nm, correlation
length 6, biases +-0.5 kT) around a 512-site bulk electrolyte; Boltzmann start, FID per
region and MSD moments recorded every step, on the mixed path (float storage, double
populations and sums). The same line carries the 256^3 single particle (radius 112,
correlation length 8) on the FP64 and the mixed path under `particle_256`.

A step is one time step of the whole sweep: hop probabilities, population, magnetisation
and moment updates, boundary handling and the per-step FP64 sums (the sweep launches and
their record finalisation, i.e. `lpc_run`). The timed region holds `lpc_run` alone, with
inputs resident in HBM; the spectrum, its peak and the diffusion coefficients are computed
on the device afterwards, their kernels warmed before, and timed on their own
(`post_ms`).

Other workloads (--workload): `particle` (the 256^3 particle alone), `batch` (512
particles of radius 8-48 in one batched sweep, against the same particles run one at a
time), `serve` (Poisson arrivals of spectrum requests through the continuous-batching
server), `equilibrate` (the population-only equilibration phase on the 256^3 particle),
`porous` (the same particle with a solid matrix, link mobility and reservoir faces),
`supercap` (the monolith / film supercapacitor study at two potentials) and `copy` (plain
device copy). Each prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Byte gap the library's arena leaves between consecutive large arrays beyond their sizes;
# the column-stream calibration carves its arrays with the same gap, so it streams the
# sweep's layout.
ARENA_STAGGER = 64 * 1024 + 256
SWEEP_SRC = os.path.join(ROOT, "paper_2603_22553_amd", "csrc", "sweep.hip")
PROFILES = os.path.join(ROOT, "profiles")
METRIC = "Glattice-site-updates/s (GSU/s) and fraction of HBM roofline"


def bytes_per_site_update(precision: str, track=("fid", "msd"), mobility: bool = False) -> int:
    """Algorithmic HBM bytes of one site-update at one step per pass: the state read once and
    written once, the fields read once. Per site the state is the population (double on both
    paths), the magnetisation (2 values) and the moments (6 values) in the storage type; the
    fields are the free energy, the per-step rotation (cos t - 1, sin t: 2 values), the region
    byte and, with link mobility, the mobility (storage type). FP64 full 169 B, mixed full 93 B,
    mixed FID-only 45 B, FP64 FID-only 73 B, FP64 populations-only 25 B."""
    s = 8 if precision == "fp64" else 4
    state = 8
    fields = s + 1
    if "fid" in track:
        state += 2 * s
        fields += 2 * s
    if "msd" in track:
        state += 6 * s
    if mobility:
        fields += s
    return 2 * state + fields


def built_bytes_per_site_update(precision: str, track=("fid", "msd"), n_regions: int = 2,
                                mobility: bool = False) -> int:
    """Bytes the kernel itself streams per site-update: it stores the phase t (one value)
    instead of the rotation pair, and reads the region byte only with more than one region."""
    s = 8 if precision == "fp64" else 4
    b = bytes_per_site_update(precision, track, mobility)
    if "fid" in track:
        b -= s
    if n_regions == 1:
        b -= 1
    return b


def sweep_source_hash() -> str:
    with open(SWEEP_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(summary: str, key: str):
    """HBM bytes per sweep launch (FETCH_SIZE + WRITE_SIZE, scaled by the copy calibration)
    from a committed rocprofv3 counter summary under profiles/, if it was taken on the
    current kernel source; otherwise None."""
    path = os.path.join(PROFILES, summary)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel source sha256\[:16\]:\s*([0-9a-f]{16})", text)
    if not m or m.group(1) != sweep_source_hash():
        return None
    m = re.search(rf"{re.escape(key)} bytes per launch:\s*([0-9.eE+]+)", text)
    return float(m.group(1)) if m else None


def roofline(n_sites, precision, ms_step, track=("fid", "msd"), traffic=None, mobility=False,
             n_regions=2):
    """Roofline object of one sweep launch (one step of n_sites sites): algorithmic bytes
    per launch over the measured time per launch, against the 8 TB/s HBM peak."""
    b = bytes_per_site_update(precision, track, mobility)
    ach = n_sites * b / (ms_step * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
            "bytes_per_site_update": b,
            "kernel_bytes_per_site_update": built_bytes_per_site_update(precision, track,
                                                                        n_regions, mobility)}


def timed(stream, fn):
    """Runs fn() between two events recorded on `stream`; returns (result, milliseconds)."""
    import torch
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    out = fn()
    t1.record(stream)
    t1.synchronize()
    torch.cuda.synchronize()
    return out, t0.elapsed_time(t1)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_timed(lat, steps, warmup, regions=(None,), msd=True):
    """Warm-up steps, one warm pass of the post-processing kernels, then `steps` steps
    timed alone (lpc_run: sweeps and record finalisation) and the post-processing timed on
    its own."""
    lat.run(warmup)

    def post():
        peaks = [lat.peak_ppm(r) for r in regions]
        return peaks, (lat.diffusion() if msd else (None, None))

    post()
    lat.synchronize()
    _, ms = timed(lat.stream, lambda: lat.run(steps))
    (peaks, (D, ratio)), ms_post = timed(lat.stream, post)
    return ms, ms_post, peaks, D, ratio


# ------------------------------------------------------------------- single large particle

def plan_for(precision, spp):
    """lpc_set_plan arguments: two steps per pass (tile code 2) or the automatic one-step
    plan."""
    return (2, 0) if spp == 2 else (0, 0)


def run_particle(f, precision, steps, warmup, track=("fid", "msd"), spp=1):
    from paper_2603_22553_amd.lattice import Lattice
    lat = Lattice(f.shape_xyz, precision=precision, track=track, n_regions=f.n_regions,
                  max_records=steps + warmup + 1)
    lat.set_plan(*plan_for(precision, spp))
    lat.set_fields(f)
    lat.init_state("uniform")
    msd = "msd" in track
    ms, ms_post, peaks, D, ratio = run_timed(lat, steps, warmup, msd=msd)
    lat.check()                    # finite FID, population conserved to 1e-12
    mass = lat.moments()[0]
    out = {"ms": ms, "post_ms": ms_post, "gsu_s": f.n_sites * steps / (ms * 1e-3) / 1e9,
           "mass_drift": float(abs(mass[-1] / mass[0] - 1.0)), "peak_ppm": peaks[0],
           "D_over_Dbulk": [round(float(v), 6) for v in ratio] if msd else None, "D": D,
           "plan": lat.describe(), "fid": lat.fid(), "uptake": lat.uptake()[-1]}
    lat.close()
    return out


def cpu_baseline(f, steps, moments=True, what="", **kw):
    """The FP64 oracle (plain C, OpenMP) timed on the host cores over `steps` steps of the
    same lattice."""
    from oracle import oracle
    oracle.build(force=False)
    t = time.perf_counter()
    oracle.run(f.F, f.delta, f.region, f.n_regions, steps, moments=moments, **kw)
    dt = time.perf_counter() - t
    tracked = "FID + MSD" if moments else "FID only"
    return {"value": round(f.n_sites * steps / dt / 1e9, 5), "unit": "GSU/s",
            "cores": oracle.threads(), "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{steps} steps of {what} (FP64, {tracked}, "
                      f"{f.n_sites * steps:.3g} site-updates), {dt:.1f} s including set-up"}


def particle_lines(f, args, precisions, track):
    """Per-precision results and roofline entries of the 256^3 particle."""
    full = track == ("fid", "msd")
    res, lines = {}, {}
    for p in precisions:
        spp = steps_per_pass(args, p)
        r = run_particle(f, p, args.steps_particle, args.warmup, track, spp)
        r["spp"] = spp
        res[p] = r
        ms_p = r["ms"] / args.steps_particle
        print(f"# particle {p}: {r['gsu_s']:.2f} GSU/s, {ms_p:.4f} ms/step, {r['plan']}",
              file=sys.stderr, flush=True)
        lines[p] = {"value": round(r["gsu_s"], 4), "unit": "GSU/s", "steps": args.steps_particle,
                    "ms_per_step": round(ms_p, 6), "post_ms": round(r["post_ms"], 3),
                    "dtype": "f64" if p == "fp64" else "f32-storage/f64-sums",
                    "roofline": roofline(f.n_sites, p, ms_p, track=track,
                                         traffic=measured_traffic(
                                             "sweep_particle_256cubed_hbm_traffic.md", p)
                                         if full else None),
                    "plan": r["plan"], "steps_per_pass": r["spp"],
                    "results": {"mass_drift": r["mass_drift"], "peak_ppm": round(r["peak_ppm"], 5),
                                "D_over_Dbulk": r["D_over_Dbulk"]}}
    if "fp64" in res and "mixed" in res:
        # the FP32-storage path against the FP64 path over the whole run (the FP64 path itself
        # is held to the oracle at 1e-10 by the parity tests)
        import numpy as np
        a, m = res["fp64"], res["mixed"]
        lines["precision_comparison"] = {
            "fid_rel_l2": float(np.linalg.norm(m["fid"] - a["fid"]) / np.linalg.norm(a["fid"])),
            "uptake_max_rel": float(np.max(np.abs(m["uptake"] - a["uptake"]) / np.abs(a["uptake"]))),
            "peak_ppm_diff": float(abs(m["peak_ppm"] - a["peak_ppm"])),
            "D_max_rel": (float(np.max(np.abs(np.asarray(m["D"]) - a["D"]) / np.abs(a["D"])))
                          if full else None),
            "steps": args.steps_particle + args.warmup}
    return lines


def steps_per_pass(args, precision):
    """Steps per sweep pass for a plain lattice: --steps-per-pass, or by default one (the
    two-step kernel is slower on MI355X: it is bound by instruction issue, not by HBM)."""
    return args.steps_per_pass or 1


def workload_particle(args):
    from paper_2603_22553_amd import synth
    f = synth.single_particle_large()
    precisions = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    track = tuple(args.track.split("+"))
    full = track == ("fid", "msd")
    args.steps_particle = args.steps
    lines = particle_lines(f, args, precisions, track)
    head = precisions[0]
    h = lines.pop(head)
    line = {
        "metric": METRIC, "value": h["value"], "unit": "GSU/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": h["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": h["dtype"], "data": "synthetic",
        "config": {"workload": "single large particle: 256^3 periodic box, radius-112 carbon "
                               "particle, " + ("FID + MSD" if full else "FID only")
                               + " recorded every step, uniform start",
                   "sites": f.n_sites, "regions": f.n_regions, "precision": head,
                   "steps_per_pass": h["steps_per_pass"], "plan": h["plan"]},
        "roofline": h["roofline"], "post_ms": h["post_ms"], "results": h["results"],
    }
    line.update(lines)
    if args.calibrate and full:
        line["calibration"] = calibration()
    if args.cpu_steps > 0:
        line["cpu_baseline"] = cpu_baseline(f, args.cpu_steps, moments=full,
                                            what="the same 256^3 particle lattice")
    return line


def calibration():
    """Achievable ceilings measured in the same run: a plain copy, and each path's sweep
    column pattern without its halo and arithmetic (256^3)."""
    cp, col, colm = copy_rate(10), columns_rate(10), columns_mixed_rate(10)
    return {"copy_GBps": round(cp, 1), "fp64_sweep_pattern_GBps": round(col, 1),
            "mixed_sweep_pattern_GBps": round(colm, 1),
            "copy_frac_of_peak": round(cp / HBM_PEAK_GBS, 4)}


# ------------------------------------------------------------------- batched particles

def workload_batch(args):
    import torch
    from paper_2603_22553_amd import synth
    from paper_2603_22553_amd.lattice import Batch, Lattice
    specs = synth.batch_specs(args.batch_count)
    t = time.perf_counter()
    fields = [synth.batch_particle(s) for s in specs]
    print(f"# generated {len(fields)} particles in {time.perf_counter() - t:.1f} s",
          file=sys.stderr, flush=True)
    sites = sum(f.n_sites for f in fields)
    steps = args.steps
    prec = "mixed"

    def make(batched):
        lats = []
        for f in fields:
            lat = Lattice(f.shape_xyz, precision=prec, n_regions=f.n_regions,
                          max_records=2 * steps + args.warmup + 1, batched=batched)
            lat.set_fields(f)
            lat.init_state("uniform")
            lats.append(lat)
        return lats

    lats = make(True)
    plans = None
    if args.tune:
        # one tuning per distinct box, timed in a batch of copies of itself
        from paper_2603_22553_amd import autotune
        t = time.perf_counter()
        plans = autotune.apply_all(lats)
        print(f"# tuned {len(plans)} box configurations in {time.perf_counter() - t:.1f} s",
              file=sys.stderr, flush=True)
    batch = Batch(lats)
    batch.run(args.warmup)
    # timed twice: launches replayed from captured graphs, then every step launched directly
    # (the second run continues the same lattices, whose record rows hold both)
    _, ms = timed(batch.stream, lambda: batch.run(steps))
    graph_desc = batch.describe()
    batch.use_graph(False)
    _, ms_direct = timed(batch.stream, lambda: batch.run(steps))
    batch.close()
    peaks = [lat.peak_ppm() for lat in lats[:4]]
    for lat in lats:
        lat.check()
        lat.close()
    torch.cuda.empty_cache()
    gsu = sites * steps / (ms * 1e-3) / 1e9
    gsu_alone = ms_alone = None
    if args.batch_alone:
        # the same particles one at a time through the single-lattice path, on the plans a
        # lattice takes when it is meant to run alone
        print("# the same particles one at a time", file=sys.stderr, flush=True)
        lats = make(False)
        for lat in lats:
            lat.run(args.warmup)

        def alone():
            for k, lat in enumerate(lats):
                lat.run(steps)
                if k % 128 == 127:
                    print(f"# queued {k + 1} lattices", file=sys.stderr, flush=True)

        _, ms_alone = timed(lats[0].stream, alone)
        for lat in lats:
            lat.close()
        gsu_alone = sites * steps / (ms_alone * 1e-3) / 1e9
    return {
        "metric": METRIC, "value": round(gsu, 4), "unit": "GSU/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": round(ms / steps, 6), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32-storage/f64-sums",
        "data": "synthetic",
        "config": {"workload": f"{len(fields)} particles, radius 8-48, box 2R+8, one batched "
                               "sweep per step, FID + MSD", "sites": sites},
        "roofline": roofline(sites, prec, ms / steps, traffic=measured_traffic(
            "sweep_batch_512particles_hbm_traffic.md", "mixed")),
        "launch": graph_desc,
        "direct_launches": {"value": round(sites * steps / (ms_direct * 1e-3) / 1e9, 4),
                            "unit": "GSU/s", "ms_per_step": round(ms_direct / steps, 6),
                            "note": "the same batch with every step launched directly"},
        "plans": ({f"{'x'.join(map(str, c[0]))}": list(v) for c, v in plans.items()}
                  if plans else "automatic (batch plans)"),
        "alone": ({"value": round(gsu_alone, 4), "unit": "GSU/s",
                   "ms_per_step": round(ms_alone / steps, 6),
                   "note": "same particles stepped one lattice at a time, on solo plans"}
                  if gsu_alone else None),
        "results": {"peak_ppm_first4": [round(p, 4) for p in peaks]},
    }


# ------------------------------------------------------------------- film

def workload_film(args):
    """The headline line: the 2048 x 256 x 256 supercapacitor film on the mixed path, with
    the 256^3 particle (FP64 and mixed) beside it."""
    from paper_2603_22553_amd import synth
    from paper_2603_22553_amd.lattice import Lattice
    t = time.perf_counter()
    f = synth.film()
    print(f"# generated film in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    steps = args.steps
    bc = ("closed", "periodic", "periodic")
    lat = Lattice(f.shape_xyz, bc=bc, precision="mixed", n_regions=3,
                  max_records=steps + args.warmup + 1)
    spp = steps_per_pass(args, "mixed")
    lat.set_plan(*plan_for("mixed", spp))
    lat.set_fields(f)
    lat.init_state("boltzmann")
    ms, ms_post, peaks, D, ratio = run_timed(lat, steps, args.warmup, regions=(0, 1, 2))
    lat.check()
    prof = lat.uptake_profile(0)
    plan = lat.describe()
    mass = lat.moments()[0]
    lat.close()
    del lat
    ms_step = ms / steps
    print(f"# film mixed: {f.n_sites * steps / (ms * 1e-3) / 1e9:.2f} GSU/s, {ms_step:.4f} ms/step, "
          f"{plan}", file=sys.stderr, flush=True)
    line = {
        "metric": METRIC, "value": round(f.n_sites * steps / (ms * 1e-3) / 1e9, 4),
        "unit": "GSU/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 6), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32-storage/f64-sums", "data": "synthetic",
        "config": {"workload": "supercapacitor film 2048x256x256: electrodes 768 | bulk 512 | "
                               "768 sites, closed in x, periodic in y and z, Boltzmann start, "
                               "FID per region + MSD recorded every step",
                   "sites": f.n_sites, "regions": 3, "precision": "mixed",
                   "steps_per_pass": spp, "plan": plan},
        "roofline": roofline(f.n_sites, "mixed", ms_step, n_regions=3,
                             traffic=measured_traffic("sweep_film_2048x256x256_hbm_traffic.md",
                                                      "mixed")),
        "post_ms": round(ms_post, 3),
        "results": {"peak_ppm_bulk_A_B": [round(p, 4) for p in peaks],
                    "D_over_Dbulk": [round(float(v), 5) for v in ratio],
                    "mass_drift": float(abs(mass[-1] / mass[0] - 1.0)),
                    "uptake_per_site_A_bulk_B": [
                        round(float(prof[:768].mean() / (256 * 256)), 5),
                        round(float(prof[768:1280].mean() / (256 * 256)), 5),
                        round(float(prof[1280:].mean() / (256 * 256)), 5)]},
    }
    if args.cpu_steps > 0:
        from oracle import oracle
        line["cpu_baseline"] = cpu_baseline(f, args.cpu_steps, what="the same film lattice",
                                            bc=(oracle.CLOSED, oracle.PERIODIC, oracle.PERIODIC),
                                            init="boltzmann")
    del f
    if args.particle_steps > 0:
        psynth = synth.single_particle_large()
        args.steps_particle = args.particle_steps
        line["particle_256"] = {
            "workload": "256^3 periodic box, radius-112 carbon particle, FID + MSD, uniform start",
            "sites": psynth.n_sites}
        line["particle_256"].update(particle_lines(psynth, args, ["fp64", "mixed"],
                                                   ("fid", "msd")))
    if args.calibrate:
        line["calibration"] = calibration()
    return line


# ------------------------------------------------------------------- porous particle, reservoirs

def workload_porous(args):
    """The extended sweep: the 256^3 particle with a quarter of its carbon sites solid
    (inaccessible), pore-width mobility on every link, and bulk reservoir faces on x
    (F = 0, rho = 1, magnetised, at 0 ppm) in place of the periodic wrap."""
    from paper_2603_22553_amd import synth
    from paper_2603_22553_amd.lattice import Lattice
    f, mu = synth.porous_particle()
    precisions = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    res = {}
    for p in precisions:
        lat = Lattice(f.shape_xyz, bc=("reservoir", "periodic", "periodic"), precision=p,
                      n_regions=f.n_regions, max_records=args.steps + args.warmup + 1,
                      mobility=True)
        lat.set_fields(f)
        lat.set_mobility(mu)
        for side in (0, 1):
            lat.set_reservoir(0, side, 0.0, 1.0, 1.0)
        lat.init_state("boltzmann")
        ms, _, peaks, D, ratio = run_timed(lat, args.steps, args.warmup)
        peak = peaks[0]
        mass = lat.moments()[0]
        plan = lat.describe()
        lat.close()
        res[p] = {"ms": ms, "gsu_s": f.n_sites * args.steps / (ms * 1e-3) / 1e9, "peak": peak,
                  "ratio": [round(float(v), 5) for v in ratio],
                  "mass_change": float(mass[-1] / mass[0] - 1.0), "plan": plan}
        print(f"# porous {p}: {res[p]['gsu_s']:.2f} GSU/s", file=sys.stderr, flush=True)
    out = None
    for p, r in res.items():
        ms_step = r["ms"] / args.steps
        # the mobility field is one more field read per site-update
        rl = roofline(f.n_sites, p, ms_step, mobility=True, n_regions=f.n_regions,
                      traffic=measured_traffic("sweep_porous_256cubed_hbm_traffic.md", p))
        entry = {"value": round(r["gsu_s"], 4), "unit": "GSU/s", "ms_per_step": round(ms_step, 6),
                 "dtype": "f64" if p == "fp64" else "f32-storage/f64-sums", "roofline": rl,
                 "results": {"peak_ppm": round(r["peak"], 4), "D_over_Dbulk": r["ratio"],
                             "mass_change": r["mass_change"]}}
        if out is None:
            out = {"metric": METRIC, "value": entry["value"], "unit": "GSU/s", "n_gpus": 1,
                   "steps": args.steps, "warmup": args.warmup,
                   "ms_per_step": entry["ms_per_step"], "higher_is_better": True,
                   "scaling": "weak", "vs_baseline": None, "dtype": entry["dtype"],
                   "data": "synthetic",
                   "config": {"workload": "porous 256^3 particle: 25 % of carbon sites solid, "
                                          "pore-width link mobility, bulk reservoir faces in x, "
                                          "Boltzmann start, FID + MSD",
                              "sites": f.n_sites, "precision": p, "plan": r["plan"]},
                   "roofline": rl, "results": entry["results"]}
        else:
            out[p] = entry
    return out


# ------------------------------------------------------------------- supercapacitor study

def workload_supercap(args):
    """The runs of section 4 with synthetic fields: monolith and film supercapacitors
    (100 x 100 x 300, electrodes of 100 planes, closed in z) at 0 V and 2 V, residence time
    1 ms, 19F at 282 MHz, mixed path; per part the spectrum peak, D / D_bulk and the uptake
    relative to 0 V. The four systems are stepped as one batch; the value is the
    site-update rate over the batched propagation."""
    from paper_2603_22553_amd import supercap
    t = time.perf_counter()
    prec = args.precision if args.precision != "both" else "mixed"
    runs, times = supercap.study(steps=args.steps, precision=prec)
    wall = time.perf_counter() - t
    su = sum(r["sites"] * r["steps"] for r in runs)
    ms = sum(times)
    ms_step = ms / args.steps                  # one batched step advances every system
    table = [{"kind": r["kind"], "potential_v": r["potential_v"],
              "parts": {k: {kk: round(vv, 5) for kk, vv in v.items()} for k, v in r["parts"].items()}}
             for r in runs]
    return {"metric": METRIC, "value": round(su / (ms * 1e-3) / 1e9, 4), "unit": "GSU/s",
            "n_gpus": 1, "steps": args.steps, "warmup": 0, "ms_per_step": round(ms_step, 6),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if prec == "fp64" else "f32-storage/f64-sums", "data": "synthetic",
            "config": {"workload": "supercapacitor study: monolith and film, 0 V and 2 V, "
                                   "100x100x300, closed in z, tau 1 ms, 282 MHz, FID + MSD, "
                                   "the four systems in one batch",
                       "runs": len(runs), "sites": runs[0]["sites"], "precision": prec},
            "roofline": roofline(sum(r["sites"] for r in runs), prec, ms_step, n_regions=3,
                                 traffic=measured_traffic(
                                     "sweep_supercap_100x100x300_hbm_traffic.md", prec)),
            "results": {"table": table, "wall_s_including_setup": round(wall, 1)}}


# ------------------------------------------------------------------- equilibration phase

def workload_equilibrate(args):
    """Equilibration phase on the 256^3 particle: populations alone, uniform start, a
    one-step-change check every --check-every steps; the threshold is 0 so exactly --steps
    steps run (the timed work does not depend on when a threshold would be met)."""
    from paper_2603_22553_amd import synth
    from paper_2603_22553_amd.lattice import Lattice
    f = synth.single_particle_large()
    precisions = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    res = {}
    for p in precisions:
        lat = Lattice(f.shape_xyz, precision=p, track=("fid", "msd"), n_regions=f.n_regions,
                      max_records=2)
        lat.set_fields(f)
        lat.init_state("uniform")
        lat.equilibrate(args.warmup, 0.0, args.check_every)
        (steps, change), ms = timed(lat.stream,
                                    lambda: lat.equilibrate(args.steps, 0.0, args.check_every))
        assert steps == args.steps
        mass = float(lat.population().sum())
        lat.close()
        res[p] = {"ms": ms, "gsu_s": f.n_sites * steps / (ms * 1e-3) / 1e9, "last_change": change,
                  "mass_drift": abs(mass / f.n_sites - 1.0)}
        print(f"# equilibrate {p}: {res[p]['gsu_s']:.2f} GSU/s", file=sys.stderr, flush=True)
    head = "fp64" if "fp64" in res else precisions[0]
    out = None
    for p, r in res.items():
        ms_step = r["ms"] / args.steps
        rl = roofline(f.n_sites, p, ms_step, track=(), n_regions=f.n_regions,
                      traffic=measured_traffic("sweep_equilibrate_256cubed_hbm_traffic.md", p))
        rl["check_bytes_per_site_update"] = round(16.0 / args.check_every, 3)
        entry = {"value": round(r["gsu_s"], 4), "unit": "GSU/s", "ms_per_step": round(ms_step, 6),
                 "dtype": "f64" if p == "fp64" else "f32-probabilities/f64-populations",
                 "roofline": rl,
                 "results": {"last_change": r["last_change"], "mass_drift": r["mass_drift"]}}
        if p == head:
            out = {"metric": METRIC, "value": entry["value"], "unit": "GSU/s", "n_gpus": 1,
                   "steps": args.steps, "warmup": args.warmup, "ms_per_step": entry["ms_per_step"],
                   "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                   "dtype": entry["dtype"], "data": "synthetic",
                   "config": {"workload": "equilibration phase on the 256^3 radius-112 particle: "
                                          "populations only, uniform start, change checked every "
                                          f"{args.check_every} steps",
                              "sites": f.n_sites, "precision": p},
                   "roofline": rl, "results": entry["results"]}
        else:
            out[p] = entry
    return out


# ------------------------------------------------------------------- serving

def _request_fields(req):
    from paper_2603_22553_amd import synth
    return synth.request_fields(req)


def generate_trace(rate, n):
    """Jobs of one trace with their inputs, generated on the host cores (worker processes
    forked before this process touches the GPU)."""
    import multiprocessing as mp
    from paper_2603_22553_amd import serve, synth
    trace = synth.serving_trace(n, rate_hz=rate)
    t = time.perf_counter()
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        fields = pool.map(_request_fields, trace, chunksize=8)
    jobs = [serve.Job(r.job_id, r.arrival_s, f, r.n_steps) for r, f in zip(trace, fields)]
    print(f"# generated {len(jobs)} requests at {rate}/s in {time.perf_counter() - t:.1f} s",
          file=sys.stderr, flush=True)
    return jobs


def serve_trace(args, rate, jobs):
    """Serves one trace of jobs: (stats, jobs)."""
    from paper_2603_22553_amd import serve
    n = len(jobs)
    ex = serve.GpuExecutor(keep_fid=True, tune=bool(args.tune_serve))
    if args.tune_serve:
        # plans of every distinct box, tuned (or read from the tuning cache) before the clock
        from paper_2603_22553_amd import autotune
        t = time.perf_counter()
        shapes = sorted({j.fields.F.shape for j in jobs})
        for nz, ny, nx in shapes:
            autotune.tune((nx, ny, nz), precision="mixed", track=("fid",), n_regions=2,
                          batched=True)
        print(f"# tuned {len(shapes)} box shapes in {time.perf_counter() - t:.1f} s",
              file=sys.stderr, flush=True)
    srv = serve.Server(ex, hbm_budget_bytes=200e9, tick_steps=args.tick_steps)
    st = srv.run(jobs, progress=lambda s: print(f"# serving {rate}/s: {s}", file=sys.stderr,
                                                 flush=True))
    su = sum(j.n_sites * j.n_steps for j in jobs)
    st["offered_gsu_s"] = su / max(max(j.arrival_s for j in jobs), 1e-9) / 1e9
    st["served_gsu_s"] = su / st["makespan_s"] / 1e9
    st["arrival_span_s"] = max(j.arrival_s for j in jobs)
    print(f"# served {n} requests at {rate}/s: {st['spectra_per_s']:.3f} spectra/s, p50 "
          f"{st['latency_p50_s']:.1f} s, p99 {st['latency_p99_s']:.1f} s", file=sys.stderr,
          flush=True)
    return st, jobs


def workload_serve(args):
    import numpy as np
    from paper_2603_22553_amd.lattice import Lattice
    rates = [float(r) for r in args.serve_rates.split(",")]
    main_rate = rates[0]
    traces = [generate_trace(main_rate, args.serve_requests)]
    traces += [generate_trace(r, args.serve_sweep_requests) for r in rates[1:]]
    import torch
    assert torch.cuda.is_available(), "no GPU"
    st, jobs = serve_trace(args, main_rate, traces[0])
    # the same first requests one at a time through the single-lattice path
    n_alone = min(len(jobs), args.serve_alone)
    t = time.perf_counter()
    su_alone = 0
    for j in jobs[:n_alone]:
        nz, ny, nx = j.fields.F.shape
        with Lattice((nx, ny, nz), precision="mixed", track=("fid",), n_regions=2,
                     max_records=j.n_steps + 1, batched=True) as lat:
            lat.set_fields(j.fields)
            lat.init_state("uniform")
            lat.run(j.n_steps)
            assert np.array_equal(lat.fid(), j.result["fid"]), "served result differs from alone"
            su_alone += j.n_sites * j.n_steps
    alone_s = time.perf_counter() - t
    r3 = lambda v: round(float(v), 3)
    out = {
        "metric": "served spectra/s with p50/p99 latency", "value": r3(st["spectra_per_s"]),
        "unit": "spectra/s", "n_gpus": 1, "steps": None, "warmup": 0,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-storage/f64-sums", "data": "synthetic",
        "config": {"workload": f"{len(jobs)} Poisson arrivals at {main_rate}/s, box sides "
                               "16-192 log-uniform, 5000-40000 steps, FID only, 200 GB budget, "
                               f"ticks of at most {args.tick_steps} steps"},
        "latency_p50_s": r3(st["latency_p50_s"]), "latency_p99_s": r3(st["latency_p99_s"]),
        "queue_p50_s": r3(st["queue_p50_s"]), "queue_p99_s": r3(st["queue_p99_s"]),
        "service_p50_s": r3(st["service_p50_s"]), "service_p99_s": r3(st["service_p99_s"]),
        "gsu_s": r3(st["served_gsu_s"]), "offered_gsu_s": r3(st["offered_gsu_s"]),
        "ticks": st["ticks"], "makespan_s": r3(st["makespan_s"]),
        "alone": {"requests": n_alone, "spectra_per_s": round(n_alone / alone_s, 4),
                  "gsu_s": r3(su_alone / alone_s / 1e9), "bitwise_equal_to_served": True},
    }
    if len(rates) > 1:
        # lower arrival rates with shorter traces: where the server keeps up, the queueing
        # delay stays bounded; the saturation throughput is the rate served at the highest load.
        # Keeping up is judged on work: the site-updates served per second over the makespan
        # against those offered per second over the arrival window (spectra per second over a
        # short trace would also count the drain after the last arrival against the rate)
        sweep = []
        for rate, tr in zip(rates[1:], traces[1:]):
            s, _ = serve_trace(args, rate, tr)
            keeps_up = (s["served_gsu_s"] >= 0.95 * s["offered_gsu_s"]
                        and s["queue_p99_s"] <= s["service_p99_s"])
            sweep.append({"rate_hz": rate, "requests": args.serve_sweep_requests,
                          "spectra_per_s": r3(s["spectra_per_s"]),
                          "latency_p50_s": r3(s["latency_p50_s"]),
                          "latency_p99_s": r3(s["latency_p99_s"]),
                          "queue_p99_s": r3(s["queue_p99_s"]),
                          "service_p99_s": r3(s["service_p99_s"]),
                          "gsu_s": r3(s["served_gsu_s"]), "offered_gsu_s": r3(s["offered_gsu_s"]),
                          "p99_bounded": bool(keeps_up)})
        out["rate_sweep"] = sweep
        bounded = [s["rate_hz"] for s in sweep if s["p99_bounded"]]
        out["highest_rate_with_bounded_p99_hz"] = max(bounded) if bounded else None
    out["saturation_spectra_per_s"] = out["value"]
    if args.serve_oracle > 0:
        # a 1 % sample of the served jobs against the oracle, over a prefix of each job's
        # steps that the oracle finishes in seconds (the served FID rows of that prefix are the
        # same records)
        from oracle import oracle
        sampled = sorted(jobs[::100], key=lambda j: j.n_sites * j.n_steps)[:args.serve_oracle]
        errs = []
        for j in sampled:
            f = j.fields
            n = min(j.n_steps, args.serve_oracle_steps)
            o = oracle.run(f.F, f.delta, f.region, f.n_regions, n, moments=False)
            g = j.result["fid"][:n + 1]
            errs.append(float(np.linalg.norm(g - o.fid()) / np.linalg.norm(o.fid())))
        out["oracle_fid_rel_l2_max"] = max(errs)
        out["oracle_sample"] = {"jobs": [j.job_id for j in sampled],
                                "steps_compared": [min(j.n_steps, args.serve_oracle_steps)
                                                   for j in sampled]}
    return out


# ------------------------------------------------------------------- copy calibration

def copy_rate(steps):
    """GB/s (read + write) of lpc_stream_copy over 1 GiB, `steps` copies timed."""
    import ctypes
    import torch
    from paper_2603_22553_amd import _native as N
    n = 1 << 30
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    s = torch.cuda.current_stream()

    def copy():
        for _ in range(steps):
            N.call("lpc_stream_copy", ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                   n, ctypes.c_void_p(s.cuda_stream))

    timed(s, copy)
    _, ms = timed(s, copy)
    assert bool(torch.equal(a[:4096], b[:4096]))
    return 2 * n * steps / (ms * 1e-3) / 1e9


def columns_rate(steps):
    """GB/s of lpc_stream_columns on 256^3: the FP64 full sweep's column streams (12 reads
    and 9 writes of doubles per site, 64 x 4 tiles, z-chunks of 128) without its halo and
    arithmetic."""
    import ctypes
    import torch
    from paper_2603_22553_amd import _native as N
    side, zc = 256, 128
    sites = side ** 3
    gap = sites + ARENA_STAGGER // 8
    buf = torch.rand(21 * gap, dtype=torch.float64, device="cuda")
    arr = [buf[k * gap:k * gap + sites] for k in range(21)]
    ins = (ctypes.c_void_p * 12)(*[t.data_ptr() for t in arr[:12]])
    outs = (ctypes.c_void_p * 9)(*[t.data_ptr() for t in arr[12:]])
    s = torch.cuda.current_stream()

    def columns():
        for _ in range(steps):
            N.call("lpc_stream_columns", ins, outs, side, side, side, zc,
                   ctypes.c_void_p(s.cuda_stream))

    timed(s, columns)
    _, ms = timed(s, columns)
    assert bool(torch.allclose(arr[12][:4096], arr[0][:4096] + (arr[9][:4096]
                               + arr[10][:4096] * arr[11][:4096]), rtol=1e-15, atol=0.0))
    return 21 * 8 * sites * steps / (ms * 1e-3) / 1e9


def columns_mixed_rate(steps):
    """GB/s of lpc_stream_columns_mixed on 256^3: the mixed full sweep's column streams
    (population in double, 10 floats and the region byte read; 9 arrays written; 89 B per
    site) without its halo and arithmetic."""
    import ctypes
    import torch
    from paper_2603_22553_amd import _native as N
    side, zc = 256, 128
    sites = side ** 3
    gap_d, gap_f = sites + ARENA_STAGGER // 8, sites + ARENA_STAGGER // 4
    rho = torch.rand(2 * gap_d, dtype=torch.float64, device="cuda")
    flt = torch.rand(18 * gap_f, dtype=torch.float32, device="cuda")
    reg = torch.randint(0, 2, (sites,), dtype=torch.uint8, device="cuda")
    f = [flt[k * gap_f:k * gap_f + sites] for k in range(18)]
    ins = (ctypes.c_void_p * 10)(*[t.data_ptr() for t in f[:10]])
    outs = (ctypes.c_void_p * 8)(*[t.data_ptr() for t in f[10:]])
    s = torch.cuda.current_stream()

    def columns():
        for _ in range(steps):
            N.call("lpc_stream_columns_mixed", ctypes.c_void_p(rho.data_ptr()), ins,
                   ctypes.c_void_p(reg.data_ptr()), ctypes.c_void_p(rho[gap_d:].data_ptr()), outs,
                   side, side, side, zc, ctypes.c_void_p(s.cuda_stream))

    timed(s, columns)
    _, ms = timed(s, columns)
    e = f[8][:4096] + f[9][:4096] * reg[:4096].float()
    assert bool(torch.allclose(f[10][:4096], f[0][:4096] + e, rtol=1e-6, atol=0.0))
    return 89 * sites * steps / (ms * 1e-3) / 1e9


def workload_copy(args):
    """Plain device copy (lpc_stream_copy) of 1 GiB: achievable HBM bandwidth, and the kernel of
    known traffic that scales the FETCH_SIZE / WRITE_SIZE counters; then the sweep's own
    column pattern (lpc_stream_columns)."""
    gbs = copy_rate(args.steps)
    gbs_c = columns_rate(args.steps)
    gbs_m = columns_mixed_rate(args.steps)
    return {"metric": "device copy bandwidth (read + write)", "value": round(gbs, 1),
            "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
            "data": "synthetic", "config": {"workload": "copy 1 GiB, lpc_stream_copy"},
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "sweep_pattern": {"GBps": round(gbs_c, 1), "frac_of_peak": round(gbs_c / HBM_PEAK_GBS, 4),
                              "frac_of_copy": round(gbs_c / gbs, 4),
                              "what": "lpc_stream_columns on 256^3: the FP64 sweep's 12 column "
                                      "reads and 9 writes per site, 64x4 tiles, zc 128, "
                                      "no halo, no arithmetic"},
            "sweep_pattern_mixed": {"GBps": round(gbs_m, 1),
                                    "frac_of_peak": round(gbs_m / HBM_PEAK_GBS, 4),
                                    "frac_of_copy": round(gbs_m / gbs, 4),
                                    "what": "lpc_stream_columns_mixed on 256^3: the mixed "
                                            "sweep's column streams, 89 B per site"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", choices=["film", "particle", "batch", "serve", "copy",
                                           "equilibrate", "porous", "supercap"],
                    default="film")
    ap.add_argument("--precision", choices=["fp64", "mixed", "both"], default="both")
    ap.add_argument("--track", choices=["fid+msd", "fid"], default="fid+msd",
                    help="particle workload: recorded quantities (fid: the serving kernel)")
    ap.add_argument("--calibrate", type=int, default=1,
                    help="film and particle workloads: also time a plain copy and the sweeps' "
                         "column patterns (achievable ceilings) and report them")
    ap.add_argument("--cpu-steps", type=int, default=None,
                    help="oracle steps timed for the CPU baseline (0 skips it; default 12 on "
                         "the film, 20 on the particle)")
    ap.add_argument("--steps-per-pass", type=int, choices=[0, 1, 2], default=0,
                    help="sweep steps per pass (temporal blocking) on the film and particle "
                         "workloads; 0: one")
    ap.add_argument("--particle-steps", type=int, default=2000,
                    help="film workload: steps of the 256^3 particle timed beside it (0 skips)")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-alone", type=int, default=1,
                    help="batch workload: also time the particles one at a time (0 skips it)")
    ap.add_argument("--tune", type=int, default=1,
                    help="batch workload: plans from the autotuner (each distinct box timed in a "
                         "batch of copies); 0: the automatic batch plans")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-rates", default="20",
                    help="comma-separated arrival rates (1/s): the first serves --serve-requests "
                         "(the headline), the others --serve-sweep-requests each")
    ap.add_argument("--serve-sweep-requests", type=int, default=300)
    ap.add_argument("--tune-serve", type=int, default=0,
                    help="serving: plans from the autotuner for every distinct box (tuned before "
                         "the clock starts)")
    ap.add_argument("--serve-alone", type=int, default=20)
    ap.add_argument("--serve-oracle", type=int, default=1,
                    help="served jobs compared with the oracle (every 100th job, cheapest first)")
    ap.add_argument("--serve-oracle-steps", type=int, default=1000,
                    help="step prefix of a sampled job that the oracle recomputes")
    ap.add_argument("--tick-steps", type=int, default=2000)
    ap.add_argument("--check-every", type=int, default=100)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the sweep "
              "would shard by slabs with one halo exchange per pass; not built).", file=sys.stderr)
        sys.exit(2)
    defaults = {"particle": (50000, 200), "batch": (2000, 20), "film": (2000, 20),
                "serve": (0, 0), "copy": (20, 1), "equilibrate": (5000, 200),
                "porous": (5000, 100), "supercap": (50000, 0)}[args.workload]
    if args.steps is None:
        args.steps = defaults[0]
    if args.warmup is None:
        args.warmup = defaults[1]
    if args.cpu_steps is None:
        args.cpu_steps = {"film": 12, "particle": 20}.get(args.workload, 0)

    if args.workload != "serve":          # serving generates its inputs before the GPU starts
        import torch
        assert torch.cuda.is_available(), "no GPU"
    fn = {"particle": workload_particle, "batch": workload_batch, "film": workload_film,
          "serve": workload_serve, "copy": workload_copy,
          "equilibrate": workload_equilibrate, "porous": workload_porous,
          "supercap": workload_supercap}[args.workload]
    print(json.dumps(fn(args)), flush=True)


if __name__ == "__main__":
    main()
