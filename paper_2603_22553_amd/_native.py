"""ctypes declarations of liblpc.so (include/lpc.h). Marshalling only.

Loading fails loudly when the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblpc.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "lpc.h")

LPC_OK, LPC_ERR_ARG, LPC_ERR_OOM, LPC_ERR_DEVICE, LPC_ERR_STATE, LPC_ERR_NONFINITE, \
    LPC_ERR_CONSERVATION = range(7)
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_OOM", 3: "ERR_DEVICE", 4: "ERR_STATE",
                5: "ERR_NONFINITE", 6: "ERR_CONSERVATION"}
BC_PERIODIC, BC_CLOSED, BC_RESERVOIR = 0, 1, 2
OPT_MOBILITY = 1
OPT_BATCHED = 2
PREC_FP64, PREC_MIXED = 0, 1
TRACK_FID, TRACK_MSD, TRACK_VACF = 1, 2, 4
INIT_UNIFORM, INIT_BOLTZMANN, INIT_USER = 0, 1, 2
MAX_REGIONS = 8


class Config(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("bc", ctypes.c_int32 * 3),
        ("precision", ctypes.c_int32),
        ("track", ctypes.c_uint32),
        ("n_regions", ctypes.c_int32),
        ("options", ctypes.c_uint32),
        ("p_hop", ctypes.c_double),
        ("dt_s", ctypes.c_double),
        ("larmor_hz", ctypes.c_double),
        ("spacing_m", ctypes.c_double),
        ("max_records", ctypes.c_int64),
        ("conservation_tol", ctypes.c_double),
    ]


class LpcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_PI64 = ctypes.POINTER(ctypes.c_int64)
_PSZ = ctypes.POINTER(ctypes.c_size_t)
_PCFG = ctypes.POINTER(Config)

SIGNATURES = {
    "lpc_config_default": [_PCFG, _I32],
    "lpc_query_footprint": [_PCFG, _PSZ],
    "lpc_create": [_PCFG, _P, _SZ, _P, ctypes.POINTER(_P)],
    "lpc_destroy": [_P],
    "lpc_set_free_energy": [_P, _P, _I64],
    "lpc_set_shift": [_P, _P, _I64],
    "lpc_set_regions": [_P, _P, _I64],
    "lpc_set_mobility": [_P, _P, _I64],
    "lpc_set_reservoir": [_P, _I32, _I32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                          ctypes.c_double],
    "lpc_init_state": [_P, _I32, _P, _I64],
    "lpc_run": [_P, _I64],
    "lpc_synchronize": [_P],
    "lpc_steps_done": [_P, _PI64],
    "lpc_record_width": [_P, ctypes.POINTER(_I32)],
    "lpc_read_records": [_P, _P, _I64, _PI64],
    "lpc_read_population": [_P, _P, _I64],
    "lpc_read_magnetization": [_P, _P, _P, _I64],
    "lpc_read_fid": [_P, _I32, _P, _P, _I64, _PI64],
    "lpc_read_moments": [_P, _P, _P, _P, _I64, _PI64],
    "lpc_read_uptake": [_P, _P, _I64, _PI64],
    "lpc_check": [_P],
    "lpc_save_state": [_P, _P, _SZ, _PSZ],
    "lpc_load_state": [_P, _P, _SZ],
    "lpc_stream_copy": [_P, _P, _SZ, _P],
    "lpc_query_linear_tiles": [_P, _P],
    "lpc_stream_columns": [_P, _P, _I32, _I32, _I32, _I32, _P],
    "lpc_stream_columns_mixed": [_P, _P, _P, _P, _P, _I32, _I32, _I32, _I32, _P],
    "lpc_describe": [_P, ctypes.c_char_p, _SZ],
    "lpc_set_plan": [_P, _I32, _I32],
    "lpc_spectrum_length": [_P, _PI64],
    "lpc_spectrum": [_P, _I32, _I64, _P, _P, _P, _I64],
    "lpc_spectrum_peak": [_P, _I32, ctypes.POINTER(ctypes.c_double)],
    "lpc_spectrum_noalloc": [_P, _I64, _I64, _P, _P],
    "lpc_diffusion": [_P, _P, _P],
    "lpc_uptake_profile": [_P, _I32, _P, _I64],
    "lpc_equilibrate": [_P, _I64, ctypes.c_double, _I64, _PI64, ctypes.POINTER(ctypes.c_double)],
    "lpc_read_vacf": [_P, _P, _I64, _PI64],
    "lpc_region_moments": [_P, _P, _I64],
    "lpc_kohn_diffusion": [_P, _I64, _P],
    "lpc_p_hop_from_residence_time": [ctypes.c_double, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_double)],
    "lpc_region_diffusion": [_P, _P, _I32, _I64, ctypes.c_double, ctypes.c_double,
                             ctypes.c_double, ctypes.c_uint32, _P, _P],
    "lpc_batch_query_footprint": [_I32, _PSZ],
    "lpc_batch_create": [_P, _I32, _P, _SZ, _P, ctypes.POINTER(_P)],
    "lpc_batch_destroy": [_P],
    "lpc_batch_run": [_P, _P],
    "lpc_batch_use_graph": [_P, _I32],
    "lpc_batch_describe": [_P, ctypes.c_char_p, _SZ],
}


def load():
    """The loaded library; raises if liblpc.so is missing (build it with build.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run paper_2603_22553_amd.build.build() "
                              "(hipcc --offload-arch=gfx950)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib.lpc_last_error.argtypes = []
        lib.lpc_last_error.restype = ctypes.c_char_p
        lib.lpc_version.argtypes = []
        lib.lpc_version.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def call(name: str, *args) -> None:
    """Calls an lpc_* function and raises LpcError with the library's message on failure."""
    lib = load()
    st = getattr(lib, name)(*args)
    if st != LPC_OK:
        raise LpcError(st, lib.lpc_last_error().decode())


def status(name: str, *args) -> int:
    """Calls an lpc_* function and returns its raw status code."""
    return getattr(load(), name)(*args)


def declared_symbols() -> list:
    """Function names declared in include/lpc.h."""
    with open(HEADER) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"\b(lpc_[a-z_]+)\s*\(", text)))
