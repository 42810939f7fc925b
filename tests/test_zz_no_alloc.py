"""lpc_spectrum_noalloc, the allocation-free variant of lpc_spectrum (its work area is a
static device array of the library): through the C ABI, its output equals lpc_spectrum's for
the same FID, on two calls in a row (the second with fewer samples, so a smaller transform
over an area that still holds the first call's values)."""
import ctypes

import numpy as np
import pytest

from paper_2603_22553_amd import _native as N
from paper_2603_22553_amd import synth

pytestmark = pytest.mark.gpu


def noalloc_spectrum(fid, n_fft=0):
    import torch
    s = torch.cuda.current_stream()
    dev = torch.from_numpy(np.ascontiguousarray(
        np.stack([fid.real, fid.imag], axis=1).reshape(-1))).cuda()
    L = n_fft or 8 * fid.size
    L = 1 << (int(L) - 1).bit_length()
    out = torch.full((2 * L,), float("nan"), dtype=torch.float64, device="cuda")
    N.call("lpc_spectrum_noalloc", ctypes.c_void_p(dev.data_ptr()), fid.size, int(n_fft),
           ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(s.cuda_stream))
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    return o[:L] + 1j * o[L:]


def test_noalloc_spectrum_equals_lattice_spectrum():
    from paper_2603_22553_amd.lattice import Lattice
    f = synth.random_fields((12, 11, 10), seed=3, delta_scale=6.0)
    for steps, n_fft in ((700, 0), (300, 0), (300, 4096)):
        with Lattice(f.shape_xyz, max_records=steps + 1) as lat:
            lat.set_fields(f)
            lat.init_state("uniform")
            lat.run(steps)
            _, want = lat.spectrum(None, n_fft=n_fft)
            fid = lat.fid()
        got = noalloc_spectrum(fid, n_fft)
        assert got.shape == want.shape
        # the same kernels on the same samples: equal to the last bit
        assert np.array_equal(got, want), (steps, n_fft, np.max(np.abs(got - want)))


def test_noalloc_spectrum_rejects_oversize():
    import torch
    fid = torch.ones(2 * 300000, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    # 8 * 300000 samples -> 2^22 points, beyond the 2^20 of the work area
    st = N.status("lpc_spectrum_noalloc", ctypes.c_void_p(fid.data_ptr()), 300000, 0,
                  ctypes.c_void_p(out.data_ptr()), None)
    assert st == N.LPC_ERR_OOM
    st = N.status("lpc_spectrum_noalloc", ctypes.c_void_p(fid.data_ptr()), 300000, 1 << 21,
                  ctypes.c_void_p(out.data_ptr()), None)
    assert st == N.LPC_ERR_OOM
    for n, L in ((0, 0), (10, 12), (10, 8)):
        st = N.status("lpc_spectrum_noalloc", ctypes.c_void_p(fid.data_ptr()), n, L,
                      ctypes.c_void_p(out.data_ptr()), None)
        assert st == N.LPC_ERR_ARG
