"""Temporal blocking: two steps per sweep pass (lpc_set_plan with LPC_TILE_TWO_STEP)
against one step per pass and against the oracle.

The two-step kernel takes the first step on 32 x 8 columns and the second on the inner
30 x 6 it owns, from first-step values kept on chip; per site the arithmetic is that of the
one-step sweep, so every state bit must equal the one-step run's, after even and odd step
counts (an odd count ends with a one-step pass). Records are summed over other tiles and
agree to rounding. The geometries cover ragged tiles in x and y (sides that are not
multiples of 30 and 6), a lattice smaller than one tile, closed and periodic faces on every
axis, degenerate axes (one or two sites, where both links of an axis reach the same site),
z-chunks of one to several planes, and up to 8 regions.
"""
import numpy as np
import pytest

from conftest import rel_l2
from paper_2603_22553_amd import _native as N
from paper_2603_22553_amd import synth

pytestmark = pytest.mark.gpu

NAMES = ("periodic", "closed")
TWO = 2                      # LPC_TILE_TWO_STEP

GEOMS = [
    # shape (x, y, z), bc (x, y, z): 0 periodic, 1 closed; precision; two-step z-chunk
    ((37, 11, 9), (0, 0, 0), "fp64", 0),
    ((37, 11, 9), (0, 0, 0), "mixed", 3),
    ((61, 13, 10), (1, 0, 1), "mixed", 4),     # closed x and z, ragged in x and y
    ((30, 6, 5), (0, 1, 0), "fp64", 2),        # exactly one tile per plane, closed y
    ((17, 5, 7), (1, 1, 1), "mixed", 1),       # smaller than a tile, all closed, zc 1
    ((1, 5, 7), (0, 0, 1), "fp64", 0),         # nx = 1
    ((2, 3, 4), (0, 1, 0), "mixed", 0),        # nx = 2: both x links reach the other site
    ((9, 1, 6), (0, 0, 0), "fp64", 2),         # ny = 1
    ((12, 7, 1), (0, 0, 0), "mixed", 0),       # nz = 1 periodic: both z links to itself
    ((12, 7, 2), (1, 0, 0), "fp64", 1),        # nz = 2, one plane per chunk
    ((64, 20, 33), (0, 0, 1), "mixed", 0),     # several chunks, closed top and bottom
]


def run(f, bc, precision, plan, steps, track=("fid", "msd"), init="boltzmann"):
    from paper_2603_22553_amd.lattice import Lattice
    with Lattice(f.shape_xyz, bc=tuple(NAMES[b] for b in bc), precision=precision, track=track,
                 n_regions=f.n_regions, max_records=steps + 1) as lat:
        lat.set_plan(*plan)
        desc = lat.describe()
        lat.set_fields(f)
        lat.init_state(init)
        lat.run(steps)
        rec = lat.records()
        blob = lat.save_state()
        out = {"records": rec, "rho": lat.population(), "desc": desc,
               "state": blob[:len(blob) - rec.size * 8]}
        if "fid" in track:
            out["m"] = lat.magnetization()
        return out


def check_records(a, b, R):
    """Records of two tilings to rounding: FID and uptake relative to their size; the drift
    sums cancel to rounding noise, so the moment columns are measured against the MSD."""
    msd = max(np.max(np.abs(b[:, 3 * R + 3:])), 1.0)
    for cols, scale in ((slice(0, 2 * R), None), (slice(2 * R, 3 * R), None),
                        (slice(3 * R, 3 * R + 6), msd)):
        x, y = a[:, cols], b[:, cols]
        assert np.max(np.abs(x - y)) <= 1e-12 * (scale or max(np.max(np.abs(y)), 1e-300))


@pytest.mark.parametrize("steps", [120, 121])
@pytest.mark.parametrize("geom", GEOMS, ids=lambda g: "x".join(map(str, g[0])) + "-" +
                         "".join("PC"[b] for b in g[1]) + "-" + g[2] + f"-zc{g[3]}")
def test_two_step_against_one_step_and_oracle(oracle, geom, steps):
    shape, bc, precision, zc = geom
    R = 3
    f = synth.random_fields(shape, seed=sum(shape) * 11 + bc[0], n_regions=R, F_scale=1.0,
                            delta_scale=6.0)
    two = run(f, bc, precision, (TWO, zc), steps)
    assert "steps per pass 2" in two["desc"]
    one = run(f, bc, precision, (0, 0), steps)
    assert "steps per pass 1" in one["desc"]
    assert two["state"] == one["state"]
    assert np.array_equal(two["rho"], one["rho"]) and np.array_equal(two["m"], one["m"])
    check_records(two["records"], one["records"], R)
    ref = oracle.run(f.F, f.delta, f.region, R, steps, bc=bc, init="boltzmann")
    rec = two["records"]
    G = rec[:, 0:2 * R:2].sum(axis=1) + 1j * rec[:, 1:2 * R:2].sum(axis=1)
    tol = 1e-10 if precision == "fp64" else 1e-4
    assert rel_l2(G, ref.fid()) <= tol
    assert np.max(np.abs(two["rho"].reshape(-1) - ref.rho)) <= tol * np.max(ref.rho)


@pytest.mark.parametrize("track", [("fid",), ("msd",), ()], ids=["fid", "msd", "rho"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_two_step_track_sets(oracle, track, precision):
    """FID-only, moments-only and population-only variants, with 1 and 8 regions."""
    for R in (1, 8):
        f = synth.random_fields((47, 19, 12), seed=5 + R, n_regions=R, F_scale=1.2)
        bc = (0, 1, 0)
        two = run(f, bc, precision, (TWO, 0), 64, track=track, init="uniform")
        one = run(f, bc, precision, (0, 0), 64, track=track, init="uniform")
        assert two["state"] == one["state"]
        check_records(two["records"], one["records"], R)
        ref = oracle.run(f.F, f.delta, f.region, R, 64, bc=bc)
        U = two["records"][:, 2 * R:3 * R]
        tol = 1e-10 if precision == "fp64" else 1e-6
        assert np.max(np.abs(U - ref.uptake())) <= tol * ref.mass()[0]


def test_two_step_plans_and_errors():
    from paper_2603_22553_amd.lattice import Lattice
    with Lattice((256, 256, 256), precision="mixed", n_regions=2, max_records=3) as lat:
        lat.set_plan(TWO, 0)
        d = lat.describe()
        # 9 x 43 tiles of 30 x 6 owned columns per plane
        assert "two-step tile 30x6" in d and "grid 9x43x" in d
        lat.set_plan(0, 0)
        assert "steps per pass 1" in lat.describe()
    with Lattice((40, 40, 40), precision="mixed", mobility=True, max_records=3) as lat:
        with pytest.raises(N.LpcError) as e:
            lat.set_plan(TWO, 0)
        assert e.value.status == N.LPC_ERR_ARG
    with Lattice((40, 40, 40), bc=("reservoir", "periodic", "periodic"), max_records=3) as lat:
        with pytest.raises(N.LpcError) as e:
            lat.set_plan(TWO, 0)
        assert e.value.status == N.LPC_ERR_ARG


def test_two_step_checkpoint_continues(oracle):
    """A run continued from a checkpoint, and runs split into odd pieces, end on the bits of
    one unbroken run."""
    f = synth.random_fields((33, 14, 9), seed=77, n_regions=2)
    from paper_2603_22553_amd.lattice import Lattice

    def make():
        lat = Lattice(f.shape_xyz, precision="mixed", n_regions=2, max_records=101)
        lat.set_plan(TWO, 2)
        lat.set_fields(f)
        lat.init_state("uniform")
        return lat

    with make() as a, make() as b:
        a.run(100)
        for k in (1, 2, 7, 3, 40, 47):
            b.run(k)
        assert np.array_equal(a.population(), b.population())
        assert np.array_equal(a.magnetization(), b.magnetization())
        assert np.array_equal(a.fid(), b.fid())


def test_full_size_particle_two_step(oracle):
    """The 256^3 particle in the benchmark's two-step plan, mixed path, over 4 steps from the
    uniform start: every state bit equal to the one-step plan, and the oracle on populations
    and every record."""
    f = synth.single_particle_large()
    steps = 4
    two = run(f, (0, 0, 0), "mixed", (TWO, 0), steps, init="uniform")
    one = run(f, (0, 0, 0), "mixed", (0, 0), steps, init="uniform")
    assert two["state"] == one["state"]
    check_records(two["records"], one["records"], 2)
    ref = oracle.run(f.F, f.delta, f.region, 2, steps)
    rec = two["records"]
    assert rel_l2(rec[:, 0] + 1j * rec[:, 1], ref.fid(0)) <= 1e-5
    assert rel_l2(rec[:, 2] + 1j * rec[:, 3], ref.fid(1)) <= 1e-5
    assert np.max(np.abs(rec[:, 4:6] - ref.uptake())) <= 1e-9 * ref.mass()[0]
    assert np.max(np.abs(two["rho"].reshape(-1) - ref.rho)) <= 1e-6
