"""Launch-plan autotuner for the lattice sweep.

For a lattice shape (with its boundaries, precision, track set and region count) it times
the sweep under each candidate plan, tile width 64 / 32 / 16 or linear tiles (where the
variant takes them) combined with the automatic z-chunk, half of it and twice it, on a
scratch lattice, and keeps the fastest. Results are
cached in a JSON file keyed by device name, ROCm version and configuration, so a shape is
timed once per machine. Any plan computes the same step (only the order of the per-step
sums changes), so tuning never changes what is computed.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import lattice as L

CACHE = os.environ.get("LPC_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "lpc_mi355x", "tune.json"))


def _key(shape_xyz, bc, precision, track, n_regions) -> str:
    dev = torch.cuda.get_device_name()
    hip = getattr(torch.version, "hip", None)
    return "|".join([dev, str(hip), "x".join(str(v) for v in shape_xyz),
                     ",".join(bc), precision, "+".join(track), f"R{n_regions}"])


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


LINEAR = 1      # tile_x of linear tiles (256 consecutive sites of the x-y plane)


def candidates(shape_xyz, auto_zc: int, linear: bool = True):
    """Candidate (tile_x, zc) plans: block widths within 1.5x of the least x padding, and
    linear tiles when `linear` (the lattice's variant takes them at this nx)."""
    nx, _, nz = shape_xyz
    pads = {tx: -(-nx // tx) * tx for tx in (64, 32, 16)}
    best_pad = min(pads.values())
    widths = [tx for tx in (64, 32, 16) if pads[tx] <= 1.5 * best_pad]
    if linear:
        widths.append(LINEAR)
    zcs = sorted({max(1, min(nz, z)) for z in (auto_zc, auto_zc // 2, 2 * auto_zc)})
    return [(tx, zc) for tx in widths for zc in zcs]


def _takes_linear(lat) -> bool:
    """Whether the lattice's sweep variant runs linear tiles at its width."""
    import ctypes
    widest = ctypes.c_int32()
    L.N.call("lpc_query_linear_tiles", ctypes.byref(lat.cfg), ctypes.byref(widest))
    return lat.shape_xyz[0] <= widest.value


def tune(shape_xyz, bc=("periodic",) * 3, precision="fp64", track=("fid", "msd"), n_regions=1,
         steps=20, warmup=3, cache_path=CACHE, use_cache=True):
    """Best (tile_x, zc) for this configuration, timed on a scratch lattice."""
    key = _key(shape_xyz, bc, precision, track, n_regions)
    cache = _load_cache(cache_path) if use_cache else {}
    if key in cache:
        v = cache[key]
        return int(v["tile_x"]), int(v["zc"])
    nx, ny, nz = shape_xyz
    rng = np.random.default_rng(0)
    probe = L.Lattice(shape_xyz, bc, precision, track, n_regions, max_records=2)
    auto_zc = probe.plan["zc"]
    linear = _takes_linear(probe)
    probe.close()
    cands = candidates(shape_xyz, auto_zc, linear)
    lat = L.Lattice(shape_xyz, bc, precision, track, n_regions,
                    max_records=len(cands) * (steps + warmup) + 1)
    lat.set_free_energy(rng.normal(0.0, 1.0, size=(nz, ny, nx)))
    lat.set_shift(rng.normal(0.0, 5.0, size=(nz, ny, nx)))
    lat.set_regions(rng.integers(0, n_regions, size=(nz, ny, nx)).astype(np.uint8))
    lat.init_state("uniform")
    timings = []
    for tx, zc in cands:
        lat.set_plan(tx, zc)
        lat.run(warmup)
        lat.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(lat.stream)
        lat.run(steps)
        t1.record(lat.stream)
        t1.synchronize()
        timings.append((t0.elapsed_time(t1) / steps, tx, zc))
    lat.close()
    ms, tx, zc = min(timings)
    if use_cache:
        cache = _load_cache(cache_path)
        cache[key] = {"tile_x": tx, "zc": zc, "ms_per_step": ms,
                      "tried": [[t, x, z] for t, x, z in timings]}
        _save_cache(cache_path, cache)
    return tx, zc


def apply(lat, **kw):
    """Tunes (or looks up) the plan for `lat`'s configuration and sets it."""
    cfg = lat.cfg
    bc = tuple("periodic" if b == 0 else "closed" for b in cfg.bc)
    precision = "fp64" if cfg.precision == 0 else "mixed"
    track = tuple(n for n, bit in (("fid", 1), ("msd", 2)) if cfg.track & bit)
    tx, zc = tune(lat.shape_xyz, bc, precision, track, lat.n_regions, **kw)
    lat.set_plan(tx, zc)
    return tx, zc
