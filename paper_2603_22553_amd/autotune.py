"""Launch-plan autotuner for the lattice sweep.

For a lattice configuration (shape, boundaries including reservoir axes, precision, track
set, regions, mobility field, batched planning) it times the sweep under each candidate plan
and keeps the fastest:
- tile widths 64 / 32 / 16 whose x padding is within 1.5x of the least, linear tiles where the
  variant takes them at this width, and two steps per pass (plain variant, lattices stepped
  alone: batches run one step per pass);
- each with the automatic z-chunk, half of it and twice it (at least 16 planes for lattices
  planned for batches).
A lattice meant to run alone is timed alone. A lattice meant for a batch is timed inside a
batch of copies of itself large enough to fill the device, since that is how its plan is
used: a small lattice alone is bound by launch latency, not by its tiles. Results are cached
in a JSON file keyed by device name, ROCm version and configuration, so a configuration is
timed once per machine. Any plan computes the same step (only the order of the per-step sums
changes), so tuning never changes what is computed.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import lattice as L

CACHE = os.environ.get("LPC_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "lpc_mi355x", "tune.json"))

LINEAR = 1      # tile_x of linear tiles (256 consecutive sites of the x-y plane)
TWO_STEP = 2    # tile_x of two steps per pass
BATCH_FILL_SITES = 32 * 1024 * 1024   # sites of the batch a batched lattice is timed in
BATCH_COPIES_MAX = 256


def _key(shape_xyz, bc, precision, track, n_regions, mobility, batched) -> str:
    dev = torch.cuda.get_device_name()
    hip = getattr(torch.version, "hip", None)
    return "|".join([dev, str(hip), "x".join(str(v) for v in shape_xyz), ",".join(bc),
                     precision, "+".join(track), f"R{n_regions}",
                     "mobility" if mobility else "plain", "batched" if batched else "alone"])


def _load_cache(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save_cache(path, data):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def candidates(shape_xyz, auto_zc: int, linear: bool = True, two_step: bool = False,
               zc_floor: int = 1):
    """Candidate (tile_x, zc) plans (zc 0: the plan's automatic z-chunk)."""
    nx, _, nz = shape_xyz
    pads = {tx: -(-nx // tx) * tx for tx in (64, 32, 16)}
    best_pad = min(pads.values())
    widths = [tx for tx in (64, 32, 16) if pads[tx] <= 1.5 * best_pad]
    if linear:
        widths.append(LINEAR)
    floor = min(nz, zc_floor)
    zcs = sorted({max(floor, min(nz, z)) for z in (auto_zc, auto_zc // 2, 2 * auto_zc)})
    out = [(tx, zc) for tx in widths for zc in zcs]
    if two_step:
        out.append((TWO_STEP, 0))
    return out


def _linear_limit(cfg) -> int:
    import ctypes
    widest = ctypes.c_int32()
    L.N.call("lpc_query_linear_tiles", ctypes.byref(cfg), ctypes.byref(widest))
    return int(widest.value)


def _probe(shape_xyz, bc, precision, track, n_regions, mobility, batched, records, seed):
    """A lattice of the configuration with random fields (and mobility, and reservoir ghosts
    on reservoir axes), initialised."""
    nx, ny, nz = shape_xyz
    rng = np.random.default_rng(seed)
    lat = L.Lattice(shape_xyz, bc, precision, track, n_regions, max_records=records,
                    mobility=mobility, batched=batched)
    lat.set_free_energy(rng.normal(0.0, 1.0, size=(nz, ny, nx)))
    lat.set_shift(rng.normal(0.0, 5.0, size=(nz, ny, nx)))
    lat.set_regions(rng.integers(0, n_regions, size=(nz, ny, nx)).astype(np.uint8))
    if mobility:
        lat.set_mobility(rng.uniform(0.2, 1.0, size=(nz, ny, nx)))
    for axis, b in enumerate(bc):
        if b == "reservoir":
            for side in (0, 1):
                lat.set_reservoir(axis, side, 0.0, 1.0, 1.0)
    lat.init_state("uniform")
    return lat


def _time(stream, fn, steps):
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    fn(steps)
    t1.record(stream)
    t1.synchronize()
    return t0.elapsed_time(t1) / steps


def tune(shape_xyz, bc=("periodic",) * 3, precision="fp64", track=("fid", "msd"), n_regions=1,
         mobility=False, batched=False, steps=20, warmup=3, cache_path=CACHE, use_cache=True):
    """Best (tile_x, zc) for this configuration, timed on scratch lattices."""
    bc = tuple(bc)
    key = _key(shape_xyz, bc, precision, track, n_regions, mobility, batched)
    cache = _load_cache(cache_path) if use_cache else {}
    if key in cache:
        v = cache[key]
        return int(v["tile_x"]), int(v["zc"])
    probe = L.Lattice(shape_xyz, bc, precision, track, n_regions, max_records=2,
                      mobility=mobility, batched=batched)
    auto_zc = probe.plan["zc"]
    linear = shape_xyz[0] <= _linear_limit(probe.cfg)
    plain = not mobility and "reservoir" not in bc
    probe.close()
    cands = candidates(shape_xyz, auto_zc, linear, two_step=plain and not batched,
                       zc_floor=16 if batched else 1)
    records = len(cands) * (steps + warmup) + 1
    sites = int(np.prod(shape_xyz))
    copies = 1
    if batched:
        copies = int(min(BATCH_COPIES_MAX, max(1, -(-BATCH_FILL_SITES // sites))))
    lats = [_probe(shape_xyz, bc, precision, track, n_regions, mobility, batched, records, k)
            for k in range(copies)]
    batch = L.Batch(lats) if batched else None
    timings = []
    try:
        for tx, zc in cands:
            for lat in lats:
                lat.set_plan(tx, zc)
            if batch is not None:
                batch.run(warmup)
                ms = _time(batch.stream, batch.run, steps)
            else:
                lats[0].run(warmup)
                ms = _time(lats[0].stream, lats[0].run, steps)
            timings.append((ms, tx, zc))
    finally:
        if batch is not None:
            batch.close()
        for lat in lats:
            lat.close()
    ms, tx, zc = min(timings)
    if use_cache:
        cache = _load_cache(cache_path)
        cache[key] = {"tile_x": tx, "zc": zc, "ms_per_step": ms, "copies": copies,
                      "tried": [[t, x, z] for t, x, z in timings]}
        _save_cache(cache_path, cache)
    return tx, zc


def config_of(lat):
    """The tuning configuration of a lattice: (shape, bc names, precision, track, regions,
    mobility, batched)."""
    cfg = lat.cfg
    names = {L.N.BC_PERIODIC: "periodic", L.N.BC_CLOSED: "closed", L.N.BC_RESERVOIR: "reservoir"}
    bc = tuple(names[int(b)] for b in cfg.bc)
    precision = "fp64" if cfg.precision == L.N.PREC_FP64 else "mixed"
    track = tuple(n for n, bit in (("fid", L.N.TRACK_FID), ("msd", L.N.TRACK_MSD))
                  if cfg.track & bit)
    mobility = bool(cfg.options & L.N.OPT_MOBILITY)
    batched = bool(cfg.options & L.N.OPT_BATCHED)
    return lat.shape_xyz, bc, precision, track, lat.n_regions, mobility, batched


def apply(lat, **kw):
    """Tunes (or looks up) the plan for `lat`'s configuration and sets it."""
    tx, zc = tune(*config_of(lat), **kw)
    lat.set_plan(tx, zc)
    return tx, zc


def apply_all(lattices, **kw):
    """Tunes each distinct configuration among `lattices` once and sets every lattice's
    plan; returns {configuration: (tile_x, zc)}."""
    plans = {}
    for lat in lattices:
        c = config_of(lat)
        if c not in plans:
            plans[c] = tune(*c, **kw)
        lat.set_plan(*plans[c])
    return plans
