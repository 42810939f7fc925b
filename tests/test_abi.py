"""C-ABI contract checks that need no GPU: the library loads, exports every function that
include/lpc.h declares, and validates configurations before touching the device."""
import ctypes
import os

import numpy as np
import pytest

from paper_2603_22553_amd import _native as N


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(N.LIB_PATH):
        from paper_2603_22553_amd import build
        build.build()
    return N.load()


def test_exports_every_declared_symbol(lib):
    names = N.declared_symbols()
    assert "lpc_run" in names and "lpc_create" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"
    # every declared call has a binding signature (or is one of the string getters)
    unbound = [n for n in names if n not in N.SIGNATURES and n not in ("lpc_last_error", "lpc_version")]
    assert not unbound


def test_version_string(lib):
    assert b"gfx950" in lib.lpc_version()


def _cfg(side=8, **kw):
    c = N.Config()
    N.call("lpc_config_default", ctypes.byref(c), side)
    for k, v in kw.items():
        if k in ("n", "bc"):
            for a in range(3):
                getattr(c, k)[a] = v[a]
        else:
            setattr(c, k, v)
    return c


def _footprint(c):
    b = ctypes.c_size_t()
    st = N.status("lpc_query_footprint", ctypes.byref(c), ctypes.byref(b))
    return st, b.value


def test_default_config(lib):
    c = _cfg(16)
    assert list(c.n) == [16, 16, 16] and list(c.bc) == [0, 0, 0]
    assert abs(c.p_hop - 1 / 7) < 1e-16 and c.dt_s == 5e-6 and c.larmor_hz == 400e6
    st, b = _footprint(c)
    assert st == N.LPC_OK and b > 0


def test_footprint_byte_model(lib):
    """The arena holds fields and two state buffers of the track set: it grows with sites,
    records and precision, and the mixed path stores the float arrays in half the space."""
    n = 64
    sites = n ** 3
    st, fp64 = _footprint(_cfg(n, max_records=1))
    st2, mixed = _footprint(_cfg(n, max_records=1, precision=N.PREC_MIXED))
    assert st == st2 == N.LPC_OK
    # per site: F, theta, region, 2 x (rho + 2 m + 6 moments); mixed: float F/theta/m/moments
    assert fp64 >= sites * (8 + 8 + 1 + 2 * 9 * 8)
    assert mixed >= sites * (4 + 4 + 1 + 2 * (8 + 8 * 4))
    assert mixed < fp64
    _, more = _footprint(_cfg(n, max_records=100001))
    assert more - fp64 >= 100000 * (3 + 6) * 8
    _, fid_only = _footprint(_cfg(n, track=N.TRACK_FID))
    assert fid_only < fp64


@pytest.mark.parametrize("field,value", [
    ("p_hop", 0.2), ("p_hop", -0.01), ("n_regions", 0), ("n_regions", 9), ("max_records", 0),
    ("precision", 5), ("track", 8), ("dt_s", 0.0), ("options", 4), ("conservation_tol", -1.0),
])
def test_config_rejected(lib, field, value):
    st, _ = _footprint(_cfg(8, **{field: value}))
    assert st == N.LPC_ERR_ARG
    assert len(lib.lpc_last_error()) > 0


def test_bad_shape_rejected(lib):
    st, _ = _footprint(_cfg(8, n=(0, 4, 4)))
    assert st == N.LPC_ERR_ARG
    st, _ = _footprint(_cfg(8, bc=(0, 3, 0)))
    assert st == N.LPC_ERR_ARG
    st, _ = _footprint(_cfg(8, bc=(0, N.BC_RESERVOIR, 0)))     # reservoir axes are valid
    assert st == N.LPC_OK


def test_mobility_field_in_footprint(lib):
    """LPC_OPT_MOBILITY adds one storage-type value per site to the arena."""
    _, plain = _footprint(_cfg(32))
    _, mob = _footprint(_cfg(32, options=N.OPT_MOBILITY))
    assert mob - plain >= 32 ** 3 * 8


def test_null_arguments(lib):
    assert N.status("lpc_query_footprint", None, None) == N.LPC_ERR_ARG
    assert N.status("lpc_destroy", None) == N.LPC_ERR_ARG
    assert N.status("lpc_run", None, 1) == N.LPC_ERR_ARG


def test_max_p_hop_accepted(lib):
    st, _ = _footprint(_cfg(4, p_hop=1.0 / 6.0))
    assert st == N.LPC_OK


def test_p_hop_from_residence_time(lib):
    """A free site is left with probability 6 p_hop per step, so its mean residence time
    is dt / (6 p_hop): the 1 ms and 0.2 ms of the paper's runs at dt = 5 us."""
    from paper_2603_22553_amd.lattice import p_hop_from_residence_time
    assert p_hop_from_residence_time(1e-3, 5e-6) == pytest.approx(1.0 / 1200.0, rel=1e-15)
    assert p_hop_from_residence_time(0.2e-3, 5e-6) == pytest.approx(1.0 / 240.0, rel=1e-15)
    # geometric stay: mean number of steps before leaving = 1 / (6 p_hop)
    p = p_hop_from_residence_time(7e-5, 5e-6)
    k = np.arange(1, 20000)
    mean_steps = np.sum(k * (1 - 6 * p) ** (k - 1) * 6 * p)
    assert mean_steps * 5e-6 == pytest.approx(7e-5, rel=1e-9)
    with pytest.raises(ValueError):
        p_hop_from_residence_time(1e-6, 5e-6)


def test_linear_tile_limits(lib):
    """Widest lattice on linear tiles per variant: the LDS window of 256 + 2 nx cells of a
    linear tile must leave two workgroups per compute unit (80 KiB each), and 2 nx halo
    sites must fit 256 threads. FP64 with FID and moments stores 88-byte cells (100 sites);
    the smaller cells reach the 128-site thread limit; mobility or reservoirs: none."""
    def limit(**kw):
        v = ctypes.c_int32(-1)
        N.call("lpc_query_linear_tiles", ctypes.byref(_cfg(8, **kw)), ctypes.byref(v))
        return v.value
    fid, msd = N.TRACK_FID, N.TRACK_MSD
    assert limit(precision=N.PREC_FP64, track=fid | msd) == 100
    assert (80 * 1024 - 1024) // 2 // 88 == 459 and (459 - 256) // 2 // 4 * 4 == 100
    assert limit(precision=N.PREC_MIXED, track=fid | msd) == 128
    assert limit(precision=N.PREC_FP64, track=fid) == 128
    assert limit(precision=N.PREC_FP64, track=0) == 128
    assert limit(precision=N.PREC_MIXED, track=fid | msd, options=N.OPT_MOBILITY) == 0
    assert limit(precision=N.PREC_FP64, track=fid | msd, options=N.OPT_BATCHED) == 100
    assert limit(precision=N.PREC_FP64, track=fid, bc=(N.BC_RESERVOIR, 0, 0)) == 0
    v = ctypes.c_int32()
    assert N.status("lpc_query_linear_tiles", ctypes.byref(_cfg(8, precision=7)),
                    ctypes.byref(v)) == N.LPC_ERR_ARG
