"""GPU-side contract of the C-ABI: error codes, ownership, determinism, checkpoints."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2603_22553_amd import _native as N
from paper_2603_22553_amd import synth

pytestmark = pytest.mark.gpu


def lattice(shape=(12, 10, 8), **kw):
    from paper_2603_22553_amd.lattice import Lattice
    kw.setdefault("max_records", 201)
    return Lattice(shape, **kw)


def test_error_codes():
    f = synth.random_fields((12, 10, 8), seed=1, n_regions=2)
    with lattice(n_regions=2) as lat:
        # run before init
        with pytest.raises(N.LpcError) as e:
            lat.run(1)
        assert e.value.status == N.LPC_ERR_STATE
        # wrong number of values
        with pytest.raises(N.LpcError) as e:
            lat.set_free_energy(np.zeros(10))
        assert e.value.status == N.LPC_ERR_ARG
        # non-finite input
        bad = f.F.copy()
        bad[3, 2, 1] = np.nan
        with pytest.raises(N.LpcError) as e:
            lat.set_free_energy(bad)
        assert e.value.status == N.LPC_ERR_NONFINITE
        bad = f.delta.copy()
        bad[0, 0, 0] = np.inf
        with pytest.raises(N.LpcError) as e:
            lat.set_shift(bad)
        assert e.value.status == N.LPC_ERR_NONFINITE
        # region id out of range
        reg = f.region.copy()
        reg[1, 1, 1] = 2
        with pytest.raises(N.LpcError) as e:
            lat.set_regions(reg)
        assert e.value.status == N.LPC_ERR_ARG
        lat.set_fields(f)
        lat.init_state("uniform")
        lat.run(150)
        # record capacity: 200 steps fit, 201 do not
        with pytest.raises(N.LpcError) as e:
            lat.run(51)
        assert e.value.status == N.LPC_ERR_STATE
        lat.run(50)
        assert lat.steps_done == 200
        with pytest.raises(N.LpcError) as e:
            lat.fid(region=2)
        assert e.value.status == N.LPC_ERR_ARG
        with pytest.raises(N.LpcError) as e:
            lat.init_state(rho=np.full(f.n_sites, np.nan))
        assert e.value.status == N.LPC_ERR_NONFINITE


def test_arena_too_small_and_misaligned():
    from paper_2603_22553_amd.lattice import make_config, footprint
    cfg = make_config((8, 8, 8), max_records=10)
    need = footprint(cfg)
    buf = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    st = N.status("lpc_create", ctypes.byref(cfg), ctypes.c_void_p(buf.data_ptr()), need - 1,
                  None, ctypes.byref(h))
    assert st == N.LPC_ERR_OOM
    st = N.status("lpc_create", ctypes.byref(cfg), ctypes.c_void_p(buf.data_ptr() + 8), need,
                  None, ctypes.byref(h))
    assert st == N.LPC_ERR_ARG


def test_arena_is_borrowed():
    """The library never frees the arena: it stays a valid torch tensor after destroy."""
    lat = lattice()
    arena = lat.arena
    lat.set_fields(synth.random_fields((12, 10, 8), seed=2))
    lat.init_state()
    lat.run(10)
    lat.close()
    arena.fill_(7)
    torch.cuda.synchronize()
    assert int(arena[0].item()) == 7


def _run(f, steps, **kw):
    with lattice(f.shape_xyz, n_regions=f.n_regions, **kw) as lat:
        lat.set_fields(f)
        lat.init_state()
        lat.run(steps)
        return lat.records(), lat.population()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bitwise_determinism(precision):
    f = synth.random_fields((40, 24, 19), seed=9, n_regions=3)
    a = _run(f, 200, precision=precision)
    b = _run(f, 200, precision=precision)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_checkpoint_restart_bitwise(precision):
    """N + M steps straight equal N steps, save, load into a fresh lattice, M steps."""
    f = synth.random_fields((20, 18, 16), seed=11, n_regions=2)
    full_rec, full_rho = _run(f, 120, precision=precision)
    with lattice(f.shape_xyz, n_regions=2, precision=precision) as a:
        a.set_fields(f)
        a.init_state()
        a.run(50)
        blob = a.save_state()
    with lattice(f.shape_xyz, n_regions=2, precision=precision) as b:
        b.set_fields(f)
        b.load_state(blob)
        assert b.steps_done == 50
        b.run(70)
        assert np.array_equal(b.records(), full_rec)
        assert np.array_equal(b.population(), full_rho)


def test_checkpoint_mismatch_rejected():
    with lattice((8, 8, 8)) as a:
        a.set_fields(synth.random_fields((8, 8, 8), seed=1))
        a.init_state()
        blob = a.save_state()
    with lattice((8, 8, 9)) as b:
        with pytest.raises(N.LpcError) as e:
            b.load_state(blob)
        assert e.value.status == N.LPC_ERR_ARG


def test_conservation_alarm_from_host_state():
    """A hand-made state whose recorded mass jumps makes the next read report it."""
    f = synth.random_fields((8, 8, 8), seed=3)
    with lattice((8, 8, 8)) as a:
        a.set_fields(f)
        a.init_state()
        a.run(5)
        blob = bytearray(a.save_state())
    # records are the tail of the checkpoint: scale the population entry of the last row
    K = 3 * 1 + 6
    tail = np.frombuffer(bytes(blob[-6 * K * 8:]), dtype=np.float64).copy().reshape(6, K)
    tail[-1, 2] *= 1.0 + 1e-9
    blob[-6 * K * 8:] = tail.tobytes()
    with lattice((8, 8, 8)) as b:
        b.set_fields(f)
        b.load_state(bytes(blob))
        with pytest.raises(N.LpcError) as e:
            b.fid()
        assert e.value.status == N.LPC_ERR_CONSERVATION
        b.records()   # raw records stay readable


def test_streams_and_async():
    """lpc_run only queues work on the lattice's stream; reads synchronize it."""
    s = torch.cuda.Stream()
    f = synth.random_fields((32, 32, 32), seed=4)
    with lattice((32, 32, 32), stream=s, max_records=1001) as lat:
        lat.set_fields(f)
        lat.init_state()
        lat.run(1000)
        rec = lat.records()
        assert rec.shape[0] == 1001 and np.all(np.isfinite(rec))


def test_plan_override_and_autotune(tmp_path):
    """Every plan computes the same step (FP64 records agree to rounding across plans and
    are bitwise equal for a repeated plan); the autotuner picks one of its candidates and
    caches it."""
    from paper_2603_22553_amd import autotune
    f = synth.random_fields((70, 20, 33), seed=21, n_regions=2)
    recs = {}
    for tx, zc in ((0, 0), (64, 5), (32, 1), (16, 33), (16, 4)):
        with lattice(f.shape_xyz, n_regions=2, max_records=101) as lat:
            lat.set_plan(tx, zc)
            if tx:
                assert lat.plan["tile_x"] == tx
            if zc:
                assert lat.plan["zc"] == zc
            lat.set_fields(f)
            lat.init_state()
            lat.run(100)
            recs[(tx, zc)] = lat.records()
    ref = recs[(0, 0)]
    for k, r in recs.items():
        assert np.max(np.abs(r - ref)) <= 1e-12 * np.max(np.abs(ref)), k
    with lattice(f.shape_xyz, n_regions=2, max_records=101) as lat:
        lat.set_plan(32, 1)
        lat.set_fields(f)
        lat.init_state()
        lat.run(100)
        assert np.array_equal(lat.records(), recs[(32, 1)])
        for bad in ((48, 0), (0, -1)):
            with pytest.raises(N.LpcError) as e:
                lat.set_plan(*bad)
            assert e.value.status == N.LPC_ERR_ARG
    cache = str(tmp_path / "tune.json")
    tx, zc = autotune.tune((70, 20, 33), n_regions=2, steps=5, cache_path=cache)
    assert tx in (64, 32, 16, autotune.LINEAR, autotune.TWO_STEP)
    assert autotune.tune((70, 20, 33), n_regions=2, steps=5, cache_path=cache) == (tx, zc)


def test_autotune_configurations(tmp_path):
    """The tuner builds its probe lattices from the target's configuration (reservoir axes,
    mobility field, batched planning), keys its cache on it, and sets plans the lattices
    take: a reservoir or mobility lattice gets a block-tile, one-step plan; a batched
    lattice is timed in a batch of copies and gets z-chunks of at least 16 planes."""
    from paper_2603_22553_amd import autotune
    from paper_2603_22553_amd.lattice import Lattice
    cache = str(tmp_path / "tune.json")
    shape = (40, 24, 36)
    with Lattice(shape, bc=("reservoir", "periodic", "closed"), n_regions=2, max_records=3) as a, \
            Lattice(shape, mobility=True, n_regions=2, max_records=3) as b, \
            Lattice(shape, precision="mixed", n_regions=2, max_records=3, batched=True) as c:
        plans = autotune.apply_all([a, b, c], steps=3, warmup=1, cache_path=cache)
        assert len(plans) == 3
        for lat in (a, b):
            assert lat.plan["tile_x"] in (64, 32, 16) and "steps per pass 1" in lat.describe()
        assert c.plan["zc"] >= 16 and "steps per pass 1" in c.describe()
    import json
    keys = list(json.load(open(cache)))
    assert any("reservoir" in k for k in keys) and any("mobility" in k for k in keys)
    assert any("batched" in k for k in keys)


def test_stream_columns_calibration():
    """lpc_stream_columns computes out[k] = in[k] + in[9] + in[10] * in[11] on a ragged
    lattice (tiles and z-chunks cut short), and rejects overlapping outputs."""
    import ctypes
    shape = (70, 9, 13)
    n = shape[0] * shape[1] * shape[2]
    buf = torch.rand(21 * n, dtype=torch.float64, device="cuda")
    arr = [buf[k * n:(k + 1) * n] for k in range(21)]
    ins = (ctypes.c_void_p * 12)(*[t.data_ptr() for t in arr[:12]])
    outs = (ctypes.c_void_p * 9)(*[t.data_ptr() for t in arr[12:]])
    s = torch.cuda.current_stream()
    N.call("lpc_stream_columns", ins, outs, *shape, 5, ctypes.c_void_p(s.cuda_stream))
    s.synchronize()
    host = buf.cpu().numpy().reshape(21, n)
    e = host[9] + host[10] * host[11]     # the kernel may fuse the product into an FMA
    for k in range(9):
        assert np.allclose(host[12 + k], host[k] + e, rtol=1e-15, atol=0.0)
    bad = (ctypes.c_void_p * 9)(*[arr[12].data_ptr()] * 9)
    with pytest.raises(N.LpcError) as err:
        N.call("lpc_stream_columns", ins, bad, *shape, 5, ctypes.c_void_p(s.cuda_stream))
    assert err.value.status == N.LPC_ERR_ARG
    with pytest.raises(N.LpcError) as err:
        N.call("lpc_stream_columns", ins, outs, *shape, 0, ctypes.c_void_p(s.cuda_stream))
    assert err.value.status == N.LPC_ERR_ARG


def test_stream_columns_mixed_calibration():
    """lpc_stream_columns_mixed computes rho_out = rho_in + e and out[k] = in[k] + e with
    e = in[8] + in[9] * region on a ragged lattice, and rejects overlapping outputs."""
    import ctypes
    shape = (70, 9, 13)
    n = shape[0] * shape[1] * shape[2]
    rho = torch.rand(2 * n, dtype=torch.float64, device="cuda")
    flt = torch.rand(18 * n, dtype=torch.float32, device="cuda")
    reg = torch.randint(0, 3, (n,), dtype=torch.uint8, device="cuda")
    f = [flt[k * n:(k + 1) * n] for k in range(18)]
    ins = (ctypes.c_void_p * 10)(*[t.data_ptr() for t in f[:10]])
    outs = (ctypes.c_void_p * 8)(*[t.data_ptr() for t in f[10:]])
    s = torch.cuda.current_stream()
    args = (ctypes.c_void_p(rho.data_ptr()), ins, ctypes.c_void_p(reg.data_ptr()),
            ctypes.c_void_p(rho[n:].data_ptr()), outs, *shape, 5, ctypes.c_void_p(s.cuda_stream))
    N.call("lpc_stream_columns_mixed", *args)
    s.synchronize()
    e = f[8].cpu().numpy() + f[9].cpu().numpy() * reg.cpu().numpy().astype(np.float32)
    r = rho.cpu().numpy()
    # e is a float that the kernel may form with one fused rounding
    assert np.allclose(r[n:], r[:n] + e.astype(np.float64), rtol=1e-6, atol=0.0)
    for k in range(8):
        assert np.allclose(f[10 + k].cpu().numpy(), f[k].cpu().numpy() + e, rtol=1e-6, atol=0.0)
    bad = (ctypes.c_void_p * 8)(*[f[10].data_ptr()] * 8)
    with pytest.raises(N.LpcError) as err:
        N.call("lpc_stream_columns_mixed", args[0], ins, args[2], args[3], bad, *shape, 5,
               ctypes.c_void_p(s.cuda_stream))
    assert err.value.status == N.LPC_ERR_ARG
