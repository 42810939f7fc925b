"""Seeded synthetic inputs for the lattice sweep: porous carbon particles and film slabs.

This module only builds input arrays (per-site free energy in kT, chemical shift in ppm,
region ids). It contains none of the sweep's arithmetic, and both the GPU path and the
CPU oracle are fed the same arrays from here.

Model inputs stand in for the paper's parametrisation (pore size -> adsorption free
energy from MD, pore size -> chemical shift from DFT, a measured pore-size distribution),
which is not available:

* A carbon particle is a ball of radius R sites centred in a cubic box of side S = 2R+8,
  so every side keeps 4 bulk sites between the particle and the box face.
* A pore-width field w (nm) over the particle comes from a Gaussian random field with a
  Gaussian correlation kernel of standard deviation `corr_len` sites, standardised over
  particle sites and mapped to widths (uniform map through the normal CDF, or lognormal).
* Inside carbon: F = -2.5 (0.7 / w) kT and delta = -6 (0.7 / w) ppm. Bulk: F = 0, delta = 0.

Arrays are C-contiguous with shape (nz, ny, nx): x is the fastest index, matching the
library's host layout.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import ndtr

W_REF_NM = 0.7          # pore width at which F = -2.5 kT and delta = -6 ppm
F_SCALE_KT = -2.5
DELTA_SCALE_PPM = -6.0
LOGNORMAL_SIGMA = 0.3   # spread of the lognormal pore-width map (an assumption; not given)


@dataclasses.dataclass
class Fields:
    """Per-site inputs of one lattice. Shapes are (nz, ny, nx)."""
    F: np.ndarray          # free energy in kT, float64
    delta: np.ndarray      # chemical shift in ppm, float64
    region: np.ndarray     # uint8 region id
    n_regions: int
    periodic: tuple = (True, True, True)   # per axis (x, y, z)

    @property
    def shape_xyz(self):
        nz, ny, nx = self.F.shape
        return (nx, ny, nz)

    @property
    def n_sites(self) -> int:
        return int(self.F.size)


def gaussian_random_field(shape, corr_len: float, rng: np.random.Generator) -> np.ndarray:
    """White noise filtered by exp(-2 pi^2 l^2 |k|^2) (k in cycles/site), periodic in every axis."""
    xi = rng.standard_normal(shape)
    spec = np.fft.rfftn(xi)
    del xi
    k2 = np.zeros(spec.shape, dtype=np.float64)
    for axis, n in enumerate(shape):
        k = np.fft.rfftfreq(n) if axis == len(shape) - 1 else np.fft.fftfreq(n)
        sh = [1] * len(shape)
        sh[axis] = k.size
        k2 = k2 + (k.reshape(sh) ** 2)
    spec *= np.exp(-2.0 * math.pi ** 2 * corr_len ** 2 * k2)
    del k2
    return np.fft.irfftn(spec, s=shape, axes=tuple(range(len(shape))))


def _standardise(g: np.ndarray, mask: np.ndarray) -> np.ndarray:
    vals = g[mask]
    if vals.size < 2:
        return np.zeros_like(g)
    sd = vals.std()
    return (g - vals.mean()) / (sd if sd > 0 else 1.0)


def width_uniform(g: np.ndarray, w_min: float, w_max: float) -> np.ndarray:
    return w_min + (w_max - w_min) * ndtr(g)


def width_lognormal(g: np.ndarray, w_med: float, sigma: float = LOGNORMAL_SIGMA) -> np.ndarray:
    return w_med * np.exp(sigma * g)


def carbon_fields(w: np.ndarray):
    """Free energy (kT) and shift (ppm) of carbon sites of pore width w (nm)."""
    r = W_REF_NM / w
    return F_SCALE_KT * r, DELTA_SCALE_PPM * r


def particle(side: int, radius: float, corr_len: float, w_range=(0.7, 2.0), seed: int = 0) -> Fields:
    """One spherical carbon particle in a periodic cubic box (region 0 bulk, 1 carbon)."""
    rng = np.random.default_rng(seed)
    shape = (side, side, side)
    c = (side - 1) / 2.0
    ax = (np.arange(side, dtype=np.float64) - c) ** 2
    r2 = ax[:, None, None] + ax[None, :, None] + ax[None, None, :]
    inside = r2 <= radius * radius
    g = _standardise(gaussian_random_field(shape, corr_len, rng), inside)
    w = width_uniform(g, *w_range)
    Fc, dc = carbon_fields(w)
    F = np.where(inside, Fc, 0.0)
    delta = np.where(inside, dc, 0.0)
    region = inside.astype(np.uint8)
    return Fields(np.ascontiguousarray(F), np.ascontiguousarray(delta), region, 2)


def single_particle_small(seed: int = 0) -> Fields:
    """32^3 periodic box, particle radius 12, correlation length 3, widths in [0.7, 2.0] nm."""
    return particle(32, 12, 3.0, (0.7, 2.0), seed)


def single_particle_large(seed: int = 1) -> Fields:
    """256^3 periodic box, particle radius 112, correlation length 8, widths in [0.7, 2.0] nm."""
    return particle(256, 112, 8.0, (0.7, 2.0), seed)


def porous_particle(side: int = 256, radius: float = 112, corr_len: float = 8.0,
                    solid_fraction: float = 0.25, w_range=(0.7, 2.0), seed: int = 1):
    """The single particle with a solid matrix and pore-size-dependent mobility.

    The carbon sites whose pore width falls in the lowest `solid_fraction` of the particle
    become inaccessible (F = +inf): the narrowest pores close first. Mobility is
    mu = w / w_max over the carbon (confined sites slower) and 1 in the bulk. Returns
    (Fields, mu).
    """
    f = particle(side, radius, corr_len, w_range, seed)
    inside = f.region == 1
    rng = np.random.default_rng(seed)
    g = _standardise(gaussian_random_field(f.F.shape, corr_len, rng), inside)
    w = width_uniform(g, *w_range)
    cut = np.quantile(w[inside], solid_fraction)
    solid = inside & (w <= cut)
    F = np.where(solid, np.inf, f.F)
    mu = np.where(inside, np.clip(w / w_range[1], 0.05, 1.0), 1.0)
    return Fields(np.ascontiguousarray(F), f.delta, f.region, f.n_regions), np.ascontiguousarray(mu)


@dataclasses.dataclass
class ParticleSpec:
    radius: int
    side: int
    w_min: float
    w_max: float
    seed: int


def batch_specs(count: int = 512, base_seed: int = 2000) -> list:
    """Radii uniform in 8..48, box side 2R+8, width range [U(0.6,1.2), U(1.5,3.0)] nm.

    The per-particle draws come from one generator seeded with (base_seed, count); the
    particle j pore field is seeded with base_seed + j.
    """
    rng = np.random.default_rng([base_seed, count])
    radii = rng.integers(8, 49, size=count)
    wmin = rng.uniform(0.6, 1.2, size=count)
    wmax = rng.uniform(1.5, 3.0, size=count)
    return [ParticleSpec(int(r), int(2 * r + 8), float(a), float(b), base_seed + j)
            for j, (r, a, b) in enumerate(zip(radii, wmin, wmax))]


def batch_particle(spec: ParticleSpec, corr_len: float = 3.0) -> Fields:
    return particle(spec.side, spec.radius, corr_len, (spec.w_min, spec.w_max), spec.seed)


def film(nx: int = 2048, ny: int = 256, nz: int = 256, elec_a: int = 768, elec_b_start: int = 1280,
         w_med_a: float = 0.9, w_med_b: float = 1.3, seed_a: int = 3, seed_b: int = 4,
         bias_a: float = 0.5, bias_b: float = -0.5, corr_len: float = 6.0) -> Fields:
    """Supercapacitor film slab along x: electrode A | bulk electrolyte | electrode B.

    Every electrode site is porous carbon (monolithic electrodes). Each electrode has its
    own lognormal pore-width field and a constant free-energy offset (bias, kT). x is
    closed (no flux through the end faces); y and z are periodic. Regions: 0 bulk, 1 A, 2 B.
    """
    F = np.zeros((nz, ny, nx), dtype=np.float64)
    delta = np.zeros_like(F)
    region = np.zeros((nz, ny, nx), dtype=np.uint8)
    for (x0, x1, w_med, seed, bias, rid) in ((0, elec_a, w_med_a, seed_a, bias_a, 1),
                                              (elec_b_start, nx, w_med_b, seed_b, bias_b, 2)):
        if x1 <= x0:
            continue
        rng = np.random.default_rng(seed)
        shape = (nz, ny, x1 - x0)
        g = gaussian_random_field(shape, corr_len, rng)
        g = (g - g.mean()) / (g.std() if g.std() > 0 else 1.0)
        w = width_lognormal(g, w_med)
        del g
        Fc, dc = carbon_fields(w)
        del w
        F[:, :, x0:x1] = Fc + bias
        delta[:, :, x0:x1] = dc
        region[:, :, x0:x1] = rid
    return Fields(F, delta, region, 3, periodic=(False, True, True))


@dataclasses.dataclass
class Request:
    """One served spectrum job."""
    job_id: int
    arrival_s: float
    side: int
    radius: int
    n_steps: int
    seed: int


def serving_trace(n_requests: int = 2000, rate_hz: float = 20.0, seed: int = 4000,
                  side_range=(16, 192), steps_range=(5000, 40000)) -> list:
    """Poisson arrivals; box sides log-uniform in side_range; step counts uniform."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    sides = np.rint(np.exp(rng.uniform(math.log(side_range[0]), math.log(side_range[1]),
                                       size=n_requests))).astype(int)
    steps = rng.integers(steps_range[0], steps_range[1] + 1, size=n_requests)
    out = []
    for j in range(n_requests):
        s = int(sides[j])
        out.append(Request(j, float(arrivals[j]), s, (s - 8) // 2, int(steps[j]), seed + 1 + j))
    return out


def request_fields(req: Request) -> Fields:
    """A served particle uses the small single-particle map (widths [0.7, 2.0], corr. length 3)."""
    return particle(req.side, req.radius, 3.0, (0.7, 2.0), req.seed)


def random_fields(shape_xyz, seed: int, F_scale: float = 1.0, delta_scale: float = 5.0,
                  n_regions: int = 1, periodic=(True, True, True)) -> Fields:
    """Unstructured random fields for small test lattices (iid normal F and delta)."""
    nx, ny, nz = shape_xyz
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((nz, ny, nx)) * F_scale
    delta = rng.standard_normal((nz, ny, nx)) * delta_scale
    region = rng.integers(0, n_regions, size=(nz, ny, nx)).astype(np.uint8)
    return Fields(F, delta, region, n_regions, tuple(periodic))
