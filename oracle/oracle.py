"""Python side of the CPU FP64 oracle. TEST INFRASTRUCTURE ONLY.

Only the tests, the entry point's smoke check and the benchmark's CPU-baseline leg use
this module. It loads `liblpc_oracle.so`, built from `lpc_oracle.c` by `build()` with the
host C compiler, and adds plain numpy post-processing of the per-step records:

* Boltzmann populations, Eq. (2): rho_i = <rho> exp(-F_i) / sum_j exp(-F_j), with the
  total equal to the number of accessible sites (the total of the uniform start).
* Inaccessible sites are those with F = +inf; every start holds nothing on them.
* FID normalised by its first sample (Eq. (8) is an average over spins).
* Spectrum, Eq. (9), by numpy's FFT (kernel exp(-2 pi i k n / L)) after zero-filling to
  the next power of two >= 8 (N+1) samples; peak by parabolic interpolation of Re F.
* Diffusion coefficient from the mean-square displacement slope over the second half of
  the run (the homogeneous limit of Eqs. (6)-(7) gives D = p0 a^2 / dt per axis).

Every parity claim of the GPU path is a comparison against what this module returns.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lpc_oracle.c")
LIB = os.path.join(HERE, "liblpc_oracle.so")

PERIODIC, CLOSED, RESERVOIR = 0, 1, 2
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with the host C compiler (plain -O2, OpenMP, no FP contraction)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-shared", "-fPIC", SRC, "-o", LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int32
        P = ctypes.c_void_p
        lib.lpc_oracle_run.argtypes = [i64, i64, i64, P, d, d, d, P, P, P, i32, P, P, P, P, P,
                                       P, P, i64, P]
        lib.lpc_oracle_run.restype = ctypes.c_int
        lib.lpc_oracle_threads.restype = ctypes.c_int
        lib.lpc_oracle_equilibrate.argtypes = [i64, i64, i64, P, d, P, P, P, P, d, i64, P, P]
        lib.lpc_oracle_equilibrate.restype = ctypes.c_int
        lib.lpc_oracle_vacf.argtypes = [i64, i64, i64, P, d, P, P, P, P, i64, P]
        lib.lpc_oracle_vacf.restype = ctypes.c_int
        _lib = lib
    return _lib


def threads() -> int:
    return int(_load().lpc_oracle_threads())


def record_width(n_regions: int) -> int:
    return 3 * n_regions + 6


def accessible(F: np.ndarray) -> np.ndarray:
    """Mask of the sites that are not part of the solid matrix (F < +inf)."""
    return ~np.isposinf(np.asarray(F, dtype=np.float64))


def boltzmann(F: np.ndarray, mean_density: float = 1.0) -> np.ndarray:
    """Eq. (2) with <rho> = mean_density per accessible site: the populations of the
    Boltzmann distribution (zero on inaccessible sites)."""
    F = np.asarray(F, dtype=np.float64)
    acc = accessible(F)
    w = np.exp(-(F - F[acc].min()))     # the common factor exp(F_min) cancels in the ratio
    return mean_density * acc.sum() * w / w.sum()


def ghosts(reservoir=None) -> np.ndarray | None:
    """Ghost values of the six faces, 4 per face (F, rho, Re m, Im m), face = 2 * axis + side
    (side 0 = low, 1 = high). `reservoir` maps (axis, side) to a tuple of those four."""
    if not reservoir:
        return None
    g = np.zeros(24)
    for (axis, side), vals in reservoir.items():
        g[4 * (2 * axis + side):4 * (2 * axis + side) + 4] = vals
    return g


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Result:
    """Per-step records plus the final state of an oracle run."""

    def __init__(self, records, n_regions, rho, re, im, M1, M2):
        self.records = records
        self.R = n_regions
        self.rho, self.re, self.im, self.M1, self.M2 = rho, re, im, M1, M2

    def fid(self, region=None) -> np.ndarray:
        R, rec = self.R, self.records
        if region is None:
            return rec[:, 0:2 * R:2].sum(axis=1) + 1j * rec[:, 1:2 * R:2].sum(axis=1)
        return rec[:, 2 * region] + 1j * rec[:, 2 * region + 1]

    def uptake(self) -> np.ndarray:
        return self.records[:, 2 * self.R:3 * self.R]

    def mass(self) -> np.ndarray:
        return self.uptake().sum(axis=1)

    def s1(self) -> np.ndarray:
        return self.records[:, 3 * self.R:3 * self.R + 3]

    def s2(self) -> np.ndarray:
        return self.records[:, 3 * self.R + 3:3 * self.R + 6]

    def msd(self) -> np.ndarray:
        return self.s2() / self.mass()[:, None]

    def drift(self) -> np.ndarray:
        return self.s1() / self.mass()[:, None]


def run(F, delta, region, n_regions, n_steps, bc=(PERIODIC, PERIODIC, PERIODIC), p0=1.0 / 7.0,
        dt=5e-6, nu0=400e6, init="uniform", moments=True, state=None, mobility=None,
        reservoir=None) -> Result:
    """Run the oracle. Arrays have shape (nz, ny, nx). init: 'uniform' (rho = m = 1 on
    accessible sites), 'boltzmann' (Eq. (2), m = rho) or an array of populations (m = rho;
    zeroed on inaccessible sites). `state` = (rho, re, im, M1, M2) continues from a saved
    state instead. `mobility`: per-site factor in [0, 1]; `reservoir`: {(axis, side): (F,
    rho, Re m, Im m)} for axes whose boundary is RESERVOIR."""
    lib = _load()
    F = np.ascontiguousarray(F, dtype=np.float64)
    acc = accessible(F).reshape(-1)
    delta = np.ascontiguousarray(delta, dtype=np.float64)
    region = np.ascontiguousarray(region, dtype=np.uint8)
    nz, ny, nx = F.shape
    n = F.size
    if state is not None:
        rho, re, im, M1, M2 = (None if a is None else np.array(a, dtype=np.float64, copy=True)
                               for a in state)
    else:
        if isinstance(init, str) and init == "uniform":
            rho = np.ones(n)
        elif isinstance(init, str) and init == "boltzmann":
            rho = boltzmann(F).reshape(-1)
        else:
            rho = np.array(init, dtype=np.float64, copy=True).reshape(-1)
        rho = np.where(acc, rho, 0.0)
        re = rho.copy()
        im = np.zeros(n)
        M1 = np.zeros(3 * n) if moments else None
        M2 = np.zeros(3 * n) if moments else None
    rho, re, im = (np.ascontiguousarray(a.reshape(-1)) for a in (rho, re, im))
    K = record_width(n_regions)
    rec = np.zeros((n_steps + 1) * K)
    bc_arr = np.asarray(bc, dtype=np.int32)
    mob = None if mobility is None else np.ascontiguousarray(mobility, dtype=np.float64).reshape(-1)
    gh = ghosts(reservoir)
    rc = lib.lpc_oracle_run(nx, ny, nz, _ptr(bc_arr), p0, dt, nu0, _ptr(F), _ptr(delta),
                            _ptr(region), n_regions, _ptr(mob), _ptr(gh), _ptr(rho), _ptr(re),
                            _ptr(im), _ptr(M1), _ptr(M2), n_steps, _ptr(rec))
    if rc != 0:
        raise RuntimeError(f"oracle failed with code {rc}")
    return Result(rec.reshape(n_steps + 1, K), n_regions, rho, re, im, M1, M2)


def equilibrate(F, n_max, tol, bc=(PERIODIC, PERIODIC, PERIODIC), p0=1.0 / 7.0, rho=None,
                mobility=None, reservoir=None):
    """Equilibration phase: populations alone stepped until the largest change in one step,
    relative to the largest population, is <= tol (or n_max steps). Returns
    (rho, steps taken, last relative change)."""
    lib = _load()
    F = np.ascontiguousarray(F, dtype=np.float64)
    nz, ny, nx = F.shape
    r = np.ones(F.size) if rho is None else np.array(rho, dtype=np.float64, copy=True).reshape(-1)
    r = np.ascontiguousarray(np.where(accessible(F).reshape(-1), r, 0.0))
    mob = None if mobility is None else np.ascontiguousarray(mobility, dtype=np.float64).reshape(-1)
    gh = ghosts(reservoir)
    steps = ctypes.c_int64()
    res = ctypes.c_double()
    bc_arr = np.asarray(bc, dtype=np.int32)
    rc = lib.lpc_oracle_equilibrate(nx, ny, nz, _ptr(bc_arr), p0, _ptr(F), _ptr(mob), _ptr(gh),
                                    _ptr(r), tol, n_max, ctypes.byref(steps), ctypes.byref(res))
    if rc != 0:
        raise RuntimeError(f"oracle equilibration failed with code {rc}")
    return r.reshape(F.shape), int(steps.value), float(res.value)


def vacf(F, n_lags, bc=(PERIODIC, PERIODIC, PERIODIC), p0=1.0 / 7.0, rho=None, mobility=None,
         reservoir=None):
    """Velocity autocorrelation of Eq. (4) by tag-field propagation: C[tau, a] =
    <dx_a(1) dx_a(1 + tau)> per particle of the start `rho` (default: Boltzmann, Eq. (2)),
    tau = 0 .. n_lags - 1. Independent of the displacement moments."""
    lib = _load()
    F = np.ascontiguousarray(F, dtype=np.float64)
    nz, ny, nx = F.shape
    r = boltzmann(F).reshape(-1) if rho is None else np.asarray(rho, dtype=np.float64).reshape(-1)
    r = np.ascontiguousarray(np.where(accessible(F).reshape(-1), r, 0.0))
    mob = None if mobility is None else np.ascontiguousarray(mobility, dtype=np.float64).reshape(-1)
    gh = ghosts(reservoir)
    C = np.zeros((n_lags, 3))
    bc_arr = np.asarray(bc, dtype=np.int32)
    rc = lib.lpc_oracle_vacf(nx, ny, nz, _ptr(bc_arr), p0, _ptr(F), _ptr(mob), _ptr(gh), _ptr(r),
                             n_lags, _ptr(C))
    if rc != 0:
        raise RuntimeError(f"oracle autocorrelation failed with code {rc}")
    return C / r.sum()


# ---------------------------------------------------------------- post-processing (Eq. (9))

def fft_length(n_samples: int) -> int:
    L = 1
    while L < 8 * n_samples:
        L *= 2
    return L


def spectrum(G: np.ndarray, dt: float, nu0: float):
    """Zero-filled FFT of the normalised FID; returns (ppm axis, complex spectrum), ppm ascending."""
    g = np.asarray(G, dtype=np.complex128) / G[0]
    L = fft_length(g.size)
    S = np.fft.fft(g, n=L)
    f = np.fft.fftfreq(L, d=dt)
    order = np.argsort(f)
    return 1e6 * f[order] / nu0, S[order]


def peak_ppm(G: np.ndarray, dt: float, nu0: float) -> float:
    """Position of the maximum of Re F, refined by a parabola through the three top bins."""
    ppm, S = spectrum(G, dt, nu0)
    y = S.real
    k = int(np.argmax(y))
    if 0 < k < y.size - 1:
        den = y[k - 1] - 2 * y[k] + y[k + 1]
        off = 0.5 * (y[k - 1] - y[k + 1]) / den if den != 0 else 0.0
    else:
        off = 0.0
    return float(ppm[k] + off * (ppm[1] - ppm[0]))


def diffusion(msd: np.ndarray, dt: float, spacing: float):
    """Per-axis D (m^2/s) from the MSD slope between step N//2 and N (lattice units^2 -> m^2)."""
    N = msd.shape[0] - 1
    h = N // 2
    slope = (msd[N] - msd[h]) / (N - h)          # lattice units^2 per step
    return spacing ** 2 * slope / (2.0 * dt), slope


def diffusion_ratio(msd: np.ndarray, p0: float) -> np.ndarray:
    """D / D_bulk: the MSD slope per step against the free-lattice slope 2 p0."""
    N = msd.shape[0] - 1
    h = N // 2
    return (msd[N] - msd[h]) / (N - h) / (2.0 * p0)
