"""Linear tiles (each workgroup steps 256 consecutive sites of the x-y plane) against the
oracle and against block tiles.

The step of Eq. (13) and the moment update are per site, so the tiling must not change
any state bit: populations, magnetisations and moments are compared bitwise between a
linear and a block plan, and records (whose summation order the tiling fixes) to rounding.
The geometries cover ragged last tiles, the widest rows each precision takes (a halo of
two rows of up to 128 sites), closed and periodic faces in every axis, and the degenerate
rows nx = 1 or ny = 1 (both links of the axis go to the site itself).
"""
import numpy as np
import pytest

from conftest import rel_l2
from paper_2603_22553_amd import _native as N
from paper_2603_22553_amd import synth

pytestmark = pytest.mark.gpu

NAMES = ("periodic", "closed")

GEOMS = [
    # shape (x, y, z), bc (x, y, z): 0 periodic, 1 closed; precision
    ((37, 11, 9), (0, 0, 0), "fp64"),      # 407 sites: 256 + a ragged tile of 151
    ((24, 24, 10), (1, 0, 1), "fp64"),     # closed x and z
    ((100, 7, 5), (0, 0, 0), "fp64"),      # the widest FP64 row: window of 256 + 200 sites
    ((100, 5, 6), (0, 1, 0), "fp64"),      # closed y
    ((128, 3, 4), (0, 0, 1), "mixed"),     # the widest mixed row, 384 sites
    ((1, 5, 7), (0, 0, 0), "fp64"),        # nx = 1
    ((2, 3, 4), (0, 1, 0), "fp64"),        # nx = 2: both x links to the other site
    ((9, 1, 6), (0, 0, 0), "fp64"),        # ny = 1
    ((16, 16, 16), (1, 1, 1), "mixed"),    # exactly one tile per plane
    ((31, 33, 8), (0, 0, 0), "mixed"),     # 1023 sites
]


def run(f, bc, precision, plan, steps, track=("fid", "msd")):
    from paper_2603_22553_amd.lattice import Lattice
    with Lattice(f.shape_xyz, bc=tuple(NAMES[b] for b in bc), precision=precision, track=track,
                 n_regions=f.n_regions, max_records=steps + 1) as lat:
        lat.set_plan(*plan)
        got = lat.plan["tile_x"]
        lat.set_fields(f)
        lat.init_state("boltzmann")
        lat.run(steps)
        rec = lat.records()
        blob = lat.save_state()
        # the checkpoint holds a header, every state array (moments included), the records
        out = {"records": rec, "rho": lat.population(), "plan": got,
               "state": blob[:len(blob) - rec.size * 8]}
        if "fid" in track:
            out["m"] = lat.magnetization()
        return out


@pytest.mark.parametrize("geom", GEOMS, ids=lambda g: "x".join(map(str, g[0])) + "-" +
                         "".join("PC"[b] for b in g[1]) + "-" + g[2])
def test_linear_tiles_against_oracle_and_blocks(oracle, geom):
    shape, bc, precision = geom
    f = synth.random_fields(shape, seed=sum(shape) * 7 + bc[1], n_regions=2, F_scale=1.0,
                            delta_scale=6.0)
    steps = 120
    lin = run(f, bc, precision, (1, 0), steps)
    assert lin["plan"] == 1
    blk = run(f, bc, precision, (16, 0), steps)
    assert blk["plan"] == 16
    # the tiling moves no state bit
    assert lin["state"] == blk["state"]
    assert np.array_equal(lin["rho"], blk["rho"])
    assert np.array_equal(lin["m"], blk["m"])
    # records to rounding: FID and uptake relative to their size; the drift sums cancel to
    # rounding noise, so both moment groups are measured against the MSD's size
    R = f.n_regions
    lr, br = lin["records"], blk["records"]
    msd = max(np.max(np.abs(br[:, 3 * R + 3:])), 1.0)
    for cols, scale in ((slice(0, 2 * R), None), (slice(2 * R, 3 * R), None),
                        (slice(3 * R, 3 * R + 6), msd)):
        a, b = lr[:, cols], br[:, cols]
        assert np.max(np.abs(a - b)) <= 1e-12 * (scale or np.max(np.abs(b)))
    ref = oracle.run(f.F, f.delta, f.region, R, steps, bc=bc, init="boltzmann")
    rec = lin["records"]
    strict = precision == "fp64"
    G = rec[:, 0:2 * R:2].sum(1) + 1j * rec[:, 1:2 * R:2].sum(1)
    assert rel_l2(G, ref.fid()) <= (1e-10 if strict else 1e-3)
    U, Uo = rec[:, 2 * R:3 * R], ref.records[:, 2 * R:3 * R]
    assert np.max(np.abs(U - Uo)) / np.max(np.abs(Uo)) <= (1e-10 if strict else 1e-5)
    S, So = rec[:, 3 * R:], ref.records[:, 3 * R:]
    assert np.max(np.abs(S - So)) / max(np.max(np.abs(So)), 1.0) <= (1e-10 if strict else 1e-4)
    er = np.max(np.abs(lin["rho"].reshape(-1) - ref.rho)) / np.max(ref.rho)
    assert er <= (1e-10 if strict else 1e-5)


@pytest.mark.parametrize("track", [("fid",), ()], ids=["fid", "population"])
def test_linear_tiles_other_track_sets(oracle, track):
    """FID-only and population-only variants on linear tiles (the widest row each takes)."""
    shape, bc = (128, 5, 7), (0, 0, 0)
    f = synth.random_fields(shape, seed=311, n_regions=2, F_scale=1.0, delta_scale=6.0)
    lin = run(f, bc, "fp64", (1, 0), 80, track=track)
    blk = run(f, bc, "fp64", (64, 0), 80, track=track)
    assert lin["state"] == blk["state"]
    assert np.array_equal(lin["rho"], blk["rho"])
    if "fid" in track:
        assert np.array_equal(lin["m"], blk["m"])
    ref = oracle.run(f.F, f.delta, f.region, 2, 80, bc=bc, init="boltzmann", moments=False)
    assert np.max(np.abs(lin["rho"].reshape(-1) - ref.rho)) <= 1e-10 * np.max(ref.rho)


# Lattices wider than a 256-site row: many block tiles per row, a ragged last tile (as
# narrow as one site), z chunks of 2 and 3 planes.
WIDE = [
    ((300, 20, 8), (1, 0, 0), "fp64"),     # 64-wide tiles: 5 per row, 32: 10, 16: 19
    ((520, 9, 6), (0, 0, 1), "mixed"),
    ((513, 5, 7), (0, 1, 0), "fp64"),      # a last tile one site wide
]


@pytest.mark.parametrize("geom", WIDE, ids=lambda g: "x".join(map(str, g[0])) + "-" +
                         "".join("PC"[b] for b in g[1]) + "-" + g[2])
def test_wide_lattices(oracle, geom):
    """Every tile of a wide lattice runs exactly once: each block width and z chunk gives
    the same state bits, the records agree to rounding and repeat bit for bit, and the
    oracle agrees."""
    shape, bc, precision = geom
    f = synth.random_fields(shape, seed=sum(shape) * 3 + bc[0], n_regions=2, F_scale=1.0,
                            delta_scale=6.0)
    steps = 60
    runs = {plan: run(f, bc, precision, plan, steps) for plan in ((64, 3), (32, 0), (16, 2))}
    again = run(f, bc, precision, (64, 3), steps)
    base = runs[(64, 3)]
    assert np.array_equal(again["records"], base["records"])
    for plan, r in runs.items():
        assert r["plan"] == plan[0]
        assert r["state"] == base["state"], plan
        assert np.array_equal(r["rho"], base["rho"]) and np.array_equal(r["m"], base["m"])
        assert np.allclose(r["records"], base["records"], rtol=1e-12,
                           atol=1e-12 * np.max(np.abs(base["records"])))
    R = f.n_regions
    ref = oracle.run(f.F, f.delta, f.region, R, steps, bc=bc, init="boltzmann")
    strict = precision == "fp64"
    rec = base["records"]
    G = rec[:, 0:2 * R:2].sum(1) + 1j * rec[:, 1:2 * R:2].sum(1)
    assert rel_l2(G, ref.fid()) <= (1e-10 if strict else 1e-3)
    er = np.max(np.abs(base["rho"].reshape(-1) - ref.rho)) / np.max(ref.rho)
    assert er <= (1e-10 if strict else 1e-5)
    S, So = rec[:, 3 * R:], ref.records[:, 3 * R:]
    assert np.max(np.abs(S - So)) / max(np.max(np.abs(So)), 1.0) <= (1e-10 if strict else 1e-4)


def test_linear_tile_choice_and_limits():
    """Automatic plans take linear tiles where they leave fewer lanes idle; linear tiles
    are refused beyond the widest row of the variant and for the extended variant."""
    from paper_2603_22553_amd.lattice import Lattice
    with Lattice((37, 11, 9), n_regions=2, max_records=2) as lat:
        assert lat.plan["tile_x"] == 1 and lat.plan["workgroups"] % 2 == 0
    with Lattice((256, 16, 8), n_regions=2, max_records=2) as lat:
        assert lat.plan["tile_x"] == 64
    with Lattice((64, 64, 8), n_regions=2, max_records=2) as lat:
        assert lat.plan["tile_x"] == 64          # no idle lane either way: block tiles
    for prec, nx in (("fp64", 101), ("mixed", 129)):
        with Lattice((nx, 3, 4), precision=prec, n_regions=2, max_records=2) as lat:
            assert lat.plan["tile_x"] != 1
            with pytest.raises(N.LpcError) as e:
                lat.set_plan(1, 0)
            assert e.value.status == N.LPC_ERR_ARG
    with Lattice((37, 11, 9), n_regions=2, max_records=2, mobility=True) as lat:
        assert lat.plan["tile_x"] != 1
        with pytest.raises(N.LpcError) as e:
            lat.set_plan(1, 0)
        assert e.value.status == N.LPC_ERR_ARG


def test_batched_lattices_plan_longer_z_chunks():
    """LPC_OPT_BATCHED: automatic plans keep z-chunks of at least 16 planes (or the whole
    axis); the step is the same (state bits equal to the default plan's)."""
    from paper_2603_22553_amd.lattice import Lattice
    f = synth.random_fields((40, 40, 64), seed=77, n_regions=2)
    out = {}
    for batched in (False, True):
        with Lattice(f.shape_xyz, n_regions=2, max_records=41, batched=batched) as lat:
            out[batched] = lat.plan["zc"]
            lat.set_fields(f)
            lat.init_state()
            lat.run(40)
            rec = lat.records()
            blob = lat.save_state()
            out[(batched, "state")] = blob[:len(blob) - rec.size * 8]
            out[(batched, "rec")] = rec
    assert out[True] >= 16 and out[False] < 16
    assert out[(True, "state")] == out[(False, "state")]
    assert np.max(np.abs(out[(True, "rec")] - out[(False, "rec")])) <= \
        1e-12 * np.max(np.abs(out[(False, "rec")]))
    with Lattice((8, 8, 9), n_regions=2, max_records=2, batched=True) as lat:
        assert lat.plan["zc"] == 9


def test_batch_mixing_linear_and_block_tiles_is_bitwise_solo():
    """A batch steps linear- and block-tiled lattices in one launch per tile kind; each
    ends as if run alone."""
    from paper_2603_22553_amd.lattice import Batch, Lattice
    shapes = [(37, 11, 9), (70, 20, 33), (24, 24, 10), (128, 3, 4)]
    fields = [synth.random_fields(s, seed=400 + k, n_regions=2) for k, s in enumerate(shapes)]
    batched = [False, True, False, True]        # default and batch-planned lattices mixed
    solo = []
    for f, bt in zip(fields, batched):
        with Lattice(f.shape_xyz, precision="mixed", n_regions=2, max_records=61,
                     batched=bt) as lat:
            lat.set_fields(f)
            lat.init_state()
            lat.run(60)
            solo.append((lat.plan["tile_x"], lat.records(), lat.population()))
    assert {p for p, _, _ in solo} >= {1, 64}
    lats = []
    try:
        for f, bt in zip(fields, batched):
            lat = Lattice(f.shape_xyz, precision="mixed", n_regions=2, max_records=61,
                          batched=bt)
            lats.append(lat)
            lat.set_fields(f)
            lat.init_state()
        b = Batch(lats)
        b.run(60)
        b.close()
        for lat, (_, rec, rho) in zip(lats, solo):
            assert np.array_equal(lat.records(), rec)
            assert np.array_equal(lat.population(), rho)
    finally:
        for lat in lats:
            lat.close()


@pytest.mark.parametrize("track", [("fid", "msd"), ("fid",)], ids=["fid+msd", "fid"])
def test_early_halo_chunks_and_widths(oracle, track):
    """Float block tiles fetch their halo two planes ahead into a third LDS buffer. Every
    z-chunk length (1, 2, 3, 5 planes and the automatic one), every block width and the
    linear tiles (one-plane halo) give the same state bits, and the oracle agrees; the
    lattice has ragged tiles in x and y and closed faces in y and z."""
    shape, bc = (70, 11, 13), (0, 1, 1)
    f = synth.random_fields(shape, seed=7013, n_regions=2, F_scale=1.0, delta_scale=6.0)
    steps = 40
    plans = [(64, 1), (64, 2), (32, 3), (16, 5), (64, 0), (1, 0)]
    runs = [run(f, bc, "mixed", plan, steps, track=track) for plan in plans]
    for plan, r in zip(plans, runs):
        assert r["plan"] == plan[0]
        assert r["state"] == runs[0]["state"], plan
        assert np.array_equal(r["rho"], runs[0]["rho"]) and np.array_equal(r["m"], runs[0]["m"])
    ref = oracle.run(f.F, f.delta, f.region, 2, steps, bc=bc, init="boltzmann",
                     moments="msd" in track)
    rec = runs[0]["records"]
    G = rec[:, 0:4:2].sum(1) + 1j * rec[:, 1:4:2].sum(1)
    assert rel_l2(G, ref.fid()) <= 1e-3
    assert np.max(np.abs(runs[0]["rho"].reshape(-1) - ref.rho)) <= 1e-5 * np.max(ref.rho)
