"""Python face of liblpc: one simulated lattice on one GPU.

A thin binding: it converts arguments, keeps the torch-allocated device arena alive and
turns status codes into exceptions. Every step of the sweep runs in the HIP library.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _native as N
from ._native import LpcError  # noqa: F401  (re-exported)

BC = {"periodic": N.BC_PERIODIC, "closed": N.BC_CLOSED, "reservoir": N.BC_RESERVOIR}
PRECISION = {"fp64": N.PREC_FP64, "mixed": N.PREC_MIXED}
INIT = {"uniform": N.INIT_UNIFORM, "boltzmann": N.INIT_BOLTZMANN, "user": N.INIT_USER}


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def p_hop_from_residence_time(tau_s: float, dt_s: float) -> float:
    """Attempt probability per neighbour for a mean residence time tau on a free site
    (lpc_p_hop_from_residence_time); raises ValueError where the library rejects the
    arguments."""
    v = ctypes.c_double()
    st = N.status("lpc_p_hop_from_residence_time", float(tau_s), float(dt_s), ctypes.byref(v))
    if st != N.LPC_OK:
        raise ValueError(N.load().lpc_last_error().decode())
    return float(v.value)


def region_diffusion(sums_a, sums_b, steps_between: int, p_hop: float, dt_s: float = 5e-6,
                     spacing_m: float = 0.5e-9, axes=(0, 1, 2)):
    """Per-region diffusion (lpc_region_diffusion) from two region-moment tables taken
    steps_between steps apart, averaged over `axes`. Returns (D in m^2/s, D / D_bulk), one
    value per region each."""
    a = np.ascontiguousarray(sums_a, dtype=np.float64).reshape(-1)
    b = np.ascontiguousarray(sums_b, dtype=np.float64).reshape(-1)
    R = a.size // 7
    if a.size != 7 * R or b.size != a.size:
        raise ValueError("region tables must hold 7 values per region, both of one size")
    D = np.empty(R)
    ratio = np.empty(R)
    mask = 0
    for ax in axes:
        mask |= 1 << int(ax)
    N.call("lpc_region_diffusion", _ptr(a), _ptr(b), R, int(steps_between), float(p_hop),
           float(dt_s), float(spacing_m), mask, _ptr(D), _ptr(ratio))
    return D, ratio


def make_config(shape_xyz, bc=("periodic",) * 3, precision="fp64", track=("fid", "msd"),
                n_regions=1, p_hop=1.0 / 7.0, dt_s=5e-6, larmor_hz=400e6, spacing_m=0.5e-9,
                max_records=1, conservation_tol=1e-12, mobility=False,
                batched=False) -> N.Config:
    cfg = N.Config()
    for a in range(3):
        cfg.n[a] = int(shape_xyz[a])
        b = bc[a]
        cfg.bc[a] = BC[b] if isinstance(b, str) else int(b)
    cfg.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    t = 0
    for name in track:
        t |= {"fid": N.TRACK_FID, "msd": N.TRACK_MSD, "vacf": N.TRACK_VACF}[name]
    cfg.track = t
    cfg.n_regions = int(n_regions)
    cfg.options = (N.OPT_MOBILITY if mobility else 0) | (N.OPT_BATCHED if batched else 0)
    cfg.p_hop = float(p_hop)
    cfg.dt_s = float(dt_s)
    cfg.larmor_hz = float(larmor_hz)
    cfg.spacing_m = float(spacing_m)
    cfg.max_records = int(max_records)
    cfg.conservation_tol = float(conservation_tol)
    return cfg


def footprint(cfg: N.Config) -> int:
    b = ctypes.c_size_t()
    N.call("lpc_query_footprint", ctypes.byref(cfg), ctypes.byref(b))
    return int(b.value)


class Lattice:
    """A lattice of nx*ny*nz sites resident in one device arena.

    shape_xyz: (nx, ny, nz); host arrays use shape (nz, ny, nx) (x fastest).
    mobility: adds the per-site mobility field. batched: plans the lattice for stepping in
    a Batch with others (longer z-chunks); solo runs then use the same plan and bits.
    """

    def __init__(self, shape_xyz, bc=("periodic",) * 3, precision="fp64", track=("fid", "msd"),
                 n_regions=1, p_hop=1.0 / 7.0, dt_s=5e-6, larmor_hz=400e6, spacing_m=0.5e-9,
                 max_records=1, conservation_tol=1e-12, device=None, stream=None,
                 mobility=False, batched=False):
        self.cfg = make_config(shape_xyz, bc, precision, track, n_regions, p_hop, dt_s,
                               larmor_hz, spacing_m, max_records, conservation_tol, mobility,
                               batched)
        self.shape_xyz = tuple(int(v) for v in shape_xyz)
        self.n_sites = int(np.prod(self.shape_xyz))
        self.n_regions = int(n_regions)
        self.track = tuple(track)
        self.device = torch.device(device if device is not None else "cuda")
        nbytes = footprint(self.cfg)
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            N.call("lpc_create", ctypes.byref(self.cfg), ctypes.c_void_p(self.arena.data_ptr()),
                   nbytes, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        self._h = h
        K = ctypes.c_int32()
        N.call("lpc_record_width", self._h, ctypes.byref(K))
        self.K = int(K.value)

    # -------------------------------------------------------------- lifetime
    @property
    def handle(self):
        if self._h is None:
            raise N.LpcError(N.LPC_ERR_STATE, "lattice is closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            N.call("lpc_destroy", self._h)
            self._h = None
            self.arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_plan(self, tile_x: int = 0, zc: int = 0):
        """Launch plan override: tile width 64/32/16, 1 for linear tiles (256 consecutive
        sites of the x-y plane; narrow lattices of the plain variant only) or 0 automatic;
        z-chunk (0 automatic)."""
        N.call("lpc_set_plan", self.handle, int(tile_x), int(zc))

    @property
    def plan(self) -> dict:
        """The launch plan as a dict (tile, zc, workgroups)."""
        import re
        d = self.describe()
        m = re.search(r"tile (\d+)x(\d+), zc (\d+), grid (\d+)x(\d+)x(\d+) = (\d+)", d)
        tx, ty, zc, gx, gy, gz, nb = (int(v) for v in m.groups())
        return {"tile_x": tx, "tile_y": ty, "zc": zc, "grid": (gx, gy, gz), "workgroups": nb}

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(512)
        N.call("lpc_describe", self.handle, buf, len(buf))
        return buf.value.decode()

    # -------------------------------------------------------------- inputs
    def _sites(self, a, dtype):
        a = np.ascontiguousarray(a, dtype=dtype).reshape(-1)
        return a

    def set_free_energy(self, F_kT):
        """Free energies in kT; +inf marks inaccessible sites (solid matrix)."""
        a = self._sites(F_kT, np.float64)
        N.call("lpc_set_free_energy", self.handle, _ptr(a), a.size)

    def set_mobility(self, mu):
        """Per-site mobility in [0, 1]; the link i-j is scaled by min(mu_i, mu_j). Needs
        mobility=True at construction."""
        a = self._sites(mu, np.float64)
        N.call("lpc_set_mobility", self.handle, _ptr(a), a.size)

    def set_reservoir(self, axis, side, F_kT=0.0, rho=0.0, m=0.0):
        """Ghost site beyond face `side` (0 low, 1 high) of a reservoir axis: free energy,
        population and complex magnetisation."""
        m = complex(m)
        N.call("lpc_set_reservoir", self.handle, int(axis), int(side), float(F_kT), float(rho),
               m.real, m.imag)

    def set_shift(self, delta_ppm):
        a = self._sites(delta_ppm, np.float64)
        N.call("lpc_set_shift", self.handle, _ptr(a), a.size)

    def set_regions(self, region):
        a = self._sites(region, np.uint8)
        N.call("lpc_set_regions", self.handle, _ptr(a), a.size)

    def set_fields(self, fields):
        """Free energy, shift and regions from a synth.Fields-like object."""
        self.set_free_energy(fields.F)
        self.set_shift(fields.delta)
        self.set_regions(fields.region)

    def init_state(self, mode="uniform", rho=None):
        if rho is not None:
            a = self._sites(rho, np.float64)
            N.call("lpc_init_state", self.handle, INIT["user"], _ptr(a), a.size)
        else:
            N.call("lpc_init_state", self.handle, INIT[mode], None, 0)

    def equilibrate(self, max_steps: int, tol: float = 1e-12, check_every: int = 100):
        """Equilibration phase: populations alone until their largest one-step change is
        <= tol relative (checked every check_every steps); then the propagation restarts
        from them (m = rho, moments 0, step 0). Returns (steps taken, last change)."""
        steps = ctypes.c_int64()
        res = ctypes.c_double()
        N.call("lpc_equilibrate", self.handle, int(max_steps), float(tol), int(check_every),
               ctypes.byref(steps), ctypes.byref(res))
        return int(steps.value), float(res.value)

    # -------------------------------------------------------------- stepping
    def run(self, n_steps: int):
        N.call("lpc_run", self.handle, int(n_steps))

    def synchronize(self):
        N.call("lpc_synchronize", self.handle)

    @property
    def steps_done(self) -> int:
        v = ctypes.c_int64()
        N.call("lpc_steps_done", self.handle, ctypes.byref(v))
        return int(v.value)

    # -------------------------------------------------------------- outputs
    def records(self) -> np.ndarray:
        rows = self.steps_done + 1
        out = np.empty((rows, self.K))
        got = ctypes.c_int64()
        N.call("lpc_read_records", self.handle, _ptr(out), rows, ctypes.byref(got))
        return out[:got.value]

    def population(self) -> np.ndarray:
        out = np.empty(self.n_sites)
        N.call("lpc_read_population", self.handle, _ptr(out), out.size)
        nx, ny, nz = self.shape_xyz
        return out.reshape(nz, ny, nx)

    def magnetization(self) -> np.ndarray:
        re = np.empty(self.n_sites)
        im = np.empty(self.n_sites)
        N.call("lpc_read_magnetization", self.handle, _ptr(re), _ptr(im), re.size)
        nx, ny, nz = self.shape_xyz
        return (re + 1j * im).reshape(nz, ny, nx)

    def fid(self, region=None) -> np.ndarray:
        rows = self.steps_done + 1
        re = np.empty(rows)
        im = np.empty(rows)
        got = ctypes.c_int64()
        N.call("lpc_read_fid", self.handle, -1 if region is None else int(region), _ptr(re),
               _ptr(im), rows, ctypes.byref(got))
        return (re + 1j * im)[:got.value]

    def moments(self):
        """(mass[rows], msd[rows, 3], drift[rows, 3]) in lattice units."""
        rows = self.steps_done + 1
        mass = np.empty(rows)
        msd = np.empty((rows, 3))
        drift = np.empty((rows, 3))
        got = ctypes.c_int64()
        N.call("lpc_read_moments", self.handle, _ptr(mass), _ptr(msd), _ptr(drift), rows,
               ctypes.byref(got))
        return mass, msd, drift

    def uptake(self) -> np.ndarray:
        rows = self.steps_done + 1
        out = np.empty((rows, self.n_regions))
        got = ctypes.c_int64()
        N.call("lpc_read_uptake", self.handle, _ptr(out), rows, ctypes.byref(got))
        return out

    # -------------------------------------------------------------- post-processing
    def spectrum(self, region=None, n_fft=0):
        """(ppm, complex spectrum) in ascending frequency, Eq. (9), computed on the device."""
        L = ctypes.c_int64()
        if n_fft == 0:
            N.call("lpc_spectrum_length", self.handle, ctypes.byref(L))
            n_fft = L.value
        ppm = np.empty(n_fft)
        re = np.empty(n_fft)
        im = np.empty(n_fft)
        N.call("lpc_spectrum", self.handle, -1 if region is None else int(region), int(n_fft),
               _ptr(ppm), _ptr(re), _ptr(im), n_fft)
        return ppm, re + 1j * im

    def peak_ppm(self, region=None) -> float:
        v = ctypes.c_double()
        N.call("lpc_spectrum_peak", self.handle, -1 if region is None else int(region),
               ctypes.byref(v))
        return float(v.value)

    def diffusion(self):
        """(D per axis in m^2/s, D / D_bulk per axis)."""
        D = np.empty(3)
        r = np.empty(3)
        N.call("lpc_diffusion", self.handle, _ptr(D), _ptr(r))
        return D, r

    def vacf(self) -> np.ndarray:
        """C(tau) = <dx_1 dx_{1+tau}> per axis, tau = 0..N-1 (Eq. (4)); runs from equilibrium."""
        n = self.steps_done
        out = np.empty((max(n, 1), 3))
        got = ctypes.c_int64()
        N.call("lpc_read_vacf", self.handle, _ptr(out), n, ctypes.byref(got))
        return out[:got.value]

    def region_moments(self) -> np.ndarray:
        """(n_regions, 7): per region the population and the M1, M2 sums along x, y, z of
        the current state."""
        out = np.empty(7 * self.n_regions)
        N.call("lpc_region_moments", self.handle, _ptr(out), out.size)
        return out.reshape(self.n_regions, 7)

    def kohn_diffusion(self, lag=None) -> np.ndarray:
        """Eq. (4) truncated at `lag` (default: all recorded lags), m^2/s per axis."""
        D = np.empty(3)
        N.call("lpc_kohn_diffusion", self.handle, -1 if lag is None else int(lag), _ptr(D))
        return D

    def uptake_profile(self, axis=0) -> np.ndarray:
        n = self.shape_xyz[axis] if 0 <= axis < 3 else 1   # the library validates the axis
        out = np.empty(n)
        N.call("lpc_uptake_profile", self.handle, int(axis), _ptr(out), n)
        return out

    def check(self):
        N.call("lpc_check", self.handle)

    # -------------------------------------------------------------- checkpoints
    def save_state(self) -> bytes:
        need = ctypes.c_size_t()
        N.call("lpc_save_state", self.handle, None, 0, ctypes.byref(need))
        buf = (ctypes.c_char * need.value)()
        got = ctypes.c_size_t()
        N.call("lpc_save_state", self.handle, buf, need.value, ctypes.byref(got))
        return bytes(buf[:got.value])

    def load_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        N.call("lpc_load_state", self.handle, buf, len(blob))


def batch_footprint(count: int) -> int:
    b = ctypes.c_size_t()
    N.call("lpc_batch_query_footprint", int(count), ctypes.byref(b))
    return int(b.value)


class Batch:
    """Lattices stepped together: one launch per step and tile width covers every lattice.

    Each lattice ends bit for bit as if it had been run alone (it keeps its own tiles and
    reduction order). The lattices must outlive the batch.
    """

    def __init__(self, lattices, stream=None, device=None):
        self.lattices = list(lattices)
        if not self.lattices:
            raise ValueError("empty batch")
        self.device = torch.device(device) if device is not None else self.lattices[0].device
        nbytes = batch_footprint(len(self.lattices))
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        handles = (ctypes.c_void_p * len(self.lattices))(*[l.handle.value for l in self.lattices])
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            N.call("lpc_batch_create", handles, len(self.lattices),
                   ctypes.c_void_p(self.arena.data_ptr()), nbytes,
                   ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        self._h = h

    def use_graph(self, enable: bool = True):
        """Replay captured graphs per chunk of steps (default) or launch every step."""
        N.call("lpc_batch_use_graph", self._h, 1 if enable else 0)

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(256)
        N.call("lpc_batch_describe", self._h, buf, len(buf))
        return buf.value.decode()

    def run(self, n_steps):
        """n_steps: one count per lattice (or a single int for all)."""
        if np.isscalar(n_steps):
            n_steps = [int(n_steps)] * len(self.lattices)
        a = np.ascontiguousarray(n_steps, dtype=np.int64)
        if a.size != len(self.lattices):
            raise ValueError("one step count per lattice")
        N.call("lpc_batch_run", self._h, _ptr(a))

    def close(self):
        if getattr(self, "_h", None) is not None:
            N.call("lpc_batch_destroy", self._h)
            self._h = None
            self.arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
