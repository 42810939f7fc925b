"""The supercapacitor study of section 4 as a workflow over the lattice library.

Two carbon electrodes in contact with bulk electrolyte, stacked along z, which is not
periodic (closed faces); x and y are periodic. Regions: 0 bulk, 1 negative electrode (low
z), 2 positive electrode (high z). Electrode structure (Fig. 7):

* ``monolith``: every electrode site is a pore of the carbon matrix;
* ``film``: monodisperse spherical carbon particles (radius 9 sites) filling 38 % of the
  electrode volume, with bulk-like sites between them.

The paper's parametrisation (MD free energies and DFT shifts of BMIM-BF4 in YP50F at 0 V
and 2 V) is not available, so the fields are synthetic stand-ins with the same roles:

* pore widths are lognormal around 0.9 nm (the most frequent sizes of section 4) on a
  correlated random field, mapped to a free energy and a shift as for the other workloads
  (``synth.carbon_fields``); bulk sites have F = 0 and no shift;
* an applied potential acts on the carbon (charged matrix) sites only: the probe anions'
  free energy there is raised by ``bias`` kT in the negative electrode and lowered by the
  same in the positive one per volt (they leave the negative electrode and accumulate in
  the positive one, Fig. 8; the bulk-like sites between film particles do not respond,
  which is why the film's uptake changes less), and the pore shifts of both electrodes
  move up by ``shift_ppm`` per volt (the higher frequencies at 2 V of Fig. 9b).

So the workflow reproduces the shape of the study (which quantities, per which part, how
they are compared), not its numbers.

Per run: Boltzmann start (Eq. (2); the closed system's exact equilibrium, so no
equilibration is needed), then propagation with the FID and the displacement moments. The
systems of a study are stepped together as one batch: a 100 x 100 x 300 lattice alone
cannot fill the GPU.
Per part it reports:

* the position of the spectrum's main peak (Eq. (9)) of the part's FID;
* D / D_bulk from the mean-square displacement slope of the particles in the part between
  the middle and the end of the run (region moments), in the plane of the electrodes (x,
  y), against the free-lattice D_bulk = p0 a^2 / dt of Eq. (7);
* the total quantity of probe anions in each electrode (Fig. 8b compares it between
  potentials).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import synth

BULK, NEGATIVE, POSITIVE = 0, 1, 2
PARTS = {BULK: "bulk", NEGATIVE: "electrode -", POSITIVE: "electrode +"}


@dataclasses.dataclass
class System:
    fields: synth.Fields
    kind: str
    potential_v: float
    carbon: np.ndarray          # (nz, ny, nx) bool: sites inside the carbon matrix


def _film_particles(shape_zyx, z0, z1, radius, fraction, rng):
    """Balls of `radius` sites at random centres that keep them inside z0 <= z < z1
    (periodic in x, y), added until their union fills `fraction` of that slab. Balls may
    touch or overlap (aggregated particles): packing 38 % without overlap is at the jamming
    limit of random sequential placement. Returns the boolean mask of particle sites."""
    nz, ny, nx = shape_zyx
    mask = np.zeros(shape_zyx, dtype=bool)
    target = fraction * (z1 - z0) * ny * nx
    r = radius
    offs = np.arange(-r, r + 1)
    dz, dy, dx = np.meshgrid(offs, offs, offs, indexing="ij")
    ball = dz ** 2 + dy ** 2 + dx ** 2 <= r * r
    dz, dy, dx = dz[ball], dy[ball], dx[ball]
    filled = 0
    while filled < target:
        cz = rng.integers(z0 + r, z1 - r)
        cy = rng.integers(0, ny)
        cx = rng.integers(0, nx)
        zz, yy, xx = cz + dz, (cy + dy) % ny, (cx + dx) % nx
        filled += int(np.count_nonzero(~mask[zz, yy, xx]))
        mask[zz, yy, xx] = True
    return mask


def system(kind: str = "monolith", potential_v: float = 0.0, shape_xyz=(100, 100, 300),
           electrode: int = 100, radius: int = 9, fraction: float = 0.38, corr_len: float = 3.0,
           w_median: float = 0.9, bias: float = 0.25, shift_ppm: float = 1.0,
           seed: int = 5000) -> System:
    """Fields of one supercapacitor: electrodes of `electrode` sites along z at both ends,
    bulk between. The carbon structure and pore field depend on `seed` only, so the two
    potentials of one seed share them."""
    if kind not in ("monolith", "film"):
        raise ValueError("kind is 'monolith' or 'film'")
    nx, ny, nz = shape_xyz
    if 2 * electrode >= nz:
        raise ValueError("the electrodes must leave bulk between them")
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    z = np.arange(nz)[:, None, None]
    region = np.where(z < electrode, NEGATIVE, np.where(z >= nz - electrode, POSITIVE, BULK))
    region = np.broadcast_to(region, shape).astype(np.uint8)
    g = synth.gaussian_random_field(shape, corr_len, rng)
    if kind == "monolith":
        carbon = region != BULK
    else:
        carbon = (_film_particles(shape, 0, electrode, radius, fraction, rng)
                  | _film_particles(shape, nz - electrode, nz, radius, fraction, rng))
    g = synth._standardise(g, carbon)
    w = synth.width_lognormal(g, w_median)
    Fc, dc = synth.carbon_fields(w)
    sign = np.where(region == NEGATIVE, 1.0, np.where(region == POSITIVE, -1.0, 0.0))
    F = np.where(carbon, Fc + potential_v * bias * sign, 0.0)
    delta = np.where(carbon, dc + potential_v * shift_ppm, 0.0)
    f = synth.Fields(np.ascontiguousarray(F), np.ascontiguousarray(delta),
                     np.ascontiguousarray(region), 3, periodic=(True, True, False))
    return System(f, kind, potential_v, carbon)


def run_batch(systems, steps: int = 50000, tau_s: float = 1e-3, dt_s: float = 5e-6,
              larmor_hz: float = 282e6, precision: str = "mixed", spacing_m: float = 0.5e-9):
    """Propagation runs of several supercapacitors on the GPU, stepped together as one
    batch (one launch per step covers every lattice, each ending bit for bit as if run
    alone); returns per-part results per system and the batch's propagation time."""
    import torch
    from .lattice import Batch, Lattice, p_hop_from_residence_time, region_diffusion
    p_hop = p_hop_from_residence_time(tau_s, dt_s)
    half = steps // 2
    lats = []
    try:
        for sysm in systems:
            f = sysm.fields
            lat = Lattice(f.shape_xyz, bc=("periodic", "periodic", "closed"),
                          precision=precision, n_regions=3, p_hop=p_hop, dt_s=dt_s,
                          larmor_hz=larmor_hz, spacing_m=spacing_m, max_records=steps + 1,
                          batched=True)
            lats.append(lat)
            lat.set_fields(f)
            lat.init_state("boltzmann")
        uptake = [lat.region_moments()[:, 0].copy() for lat in lats]
        batch = Batch(lats)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(batch.stream)
        batch.run(half)
        mom_a = [lat.region_moments() for lat in lats]
        batch.run(steps - half)
        t1.record(batch.stream)
        mom_b = [lat.region_moments() for lat in lats]
        t1.synchronize()
        ms = t0.elapsed_time(t1)
        batch.close()
        out = []
        for sysm, lat, up, ma, mb in zip(systems, lats, uptake, mom_a, mom_b):
            peaks = [lat.peak_ppm(r) for r in range(3)]
            lat.check()
            # in the electrode plane (x, y); z is closed at the electrode backs
            _, ratio = region_diffusion(ma, mb, steps - half, p_hop, dt_s, spacing_m,
                                        axes=(0, 1))
            out.append({"kind": sysm.kind, "potential_v": sysm.potential_v, "tau_s": tau_s,
                        "p_hop": p_hop, "steps": steps, "sites": sysm.fields.n_sites,
                        "parts": {PARTS[r]: {"peak_ppm": float(peaks[r]),
                                             "D_over_Dbulk": float(ratio[r]),
                                             "uptake": float(up[r])} for r in range(3)}})
        return out, ms
    finally:
        for lat in lats:
            lat.close()


def run(sysm: System, steps: int = 50000, tau_s: float = 1e-3, dt_s: float = 5e-6,
        larmor_hz: float = 282e6, precision: str = "mixed", spacing_m: float = 0.5e-9):
    """One propagation run of a supercapacitor on the GPU; returns per-part results."""
    out, ms = run_batch([sysm], steps, tau_s, dt_s, larmor_hz, precision, spacing_m)
    out[0]["propagate_ms"] = ms
    return out[0]


def study(kinds=("monolith", "film"), potentials=(0.0, 2.0), taus=(1e-3,), steps: int = 50000,
          shape_xyz=(100, 100, 300), electrode: int = 100, precision: str = "mixed",
          seed: int = 5000, **system_kw):
    """The runs of section 4 for every (structure, potential, residence time), the systems
    of one residence time stepped as one batch, plus the normalised electrode uptake
    rho_tot(V) / rho_tot(0 V) of Fig. 8b per structure. Returns (runs, propagation ms per
    batch)."""
    systems = [system(kind, v, shape_xyz, electrode, seed=seed, **system_kw)
               for kind in kinds for v in potentials]
    runs, times = [], []
    for tau in taus:
        out, ms = run_batch(systems, steps, tau, precision=precision)
        runs.extend(out)
        times.append(ms)
    base = {r["kind"]: r for r in runs if r["potential_v"] == 0.0 and r["tau_s"] == taus[0]}
    for r in runs:
        b = base.get(r["kind"])
        if b is None:
            continue
        for part in ("electrode -", "electrode +"):
            r["parts"][part]["uptake_vs_0V"] = (r["parts"][part]["uptake"]
                                                / b["parts"][part]["uptake"])
    return runs, times
