"""Inaccessible sites, link mobility and reservoir faces on the GPU path, against the oracle.

Section 2.1 and Fig. 1 (moves towards the solid matrix are rejected), the passage after
Eq. (7) (a symmetric factor per link), section 3.2 (Dirichlet ghost layers on non-periodic
boundaries). Tolerances as for the plain sweep: FP64 records within 1e-10, mixed FID
relative L2 within 1e-3; totals are compared to the oracle's instead of being held
constant, since reservoir faces exchange matter.
"""
import math

import numpy as np
import pytest

from conftest import rel_l2
from paper_2603_22553_amd import synth

pytestmark = pytest.mark.gpu

PER, CLO, RES = 0, 1, 2
NAMES = {PER: "periodic", CLO: "closed", RES: "reservoir"}
INF = math.inf


def scene(shape_xyz, seed, obstacles=0.2, mobility=False, bc=(PER, PER, PER), n_regions=2):
    """Random fields with a share of inaccessible sites, optional mobility and random
    magnetised ghosts on the reservoir faces."""
    f = synth.random_fields(shape_xyz, seed=seed, n_regions=n_regions, F_scale=1.0,
                            delta_scale=6.0)
    rng = np.random.default_rng(seed + 1000)
    mask = rng.random(f.F.shape) < obstacles
    F = np.where(mask, INF, f.F)
    mu = rng.uniform(0.1, 1.0, size=f.F.shape) if mobility else None
    faces = {}
    for axis in range(3):
        if bc[axis] == RES:
            for side in (0, 1):
                faces[(axis, side)] = (rng.normal(0.0, 1.0), rng.uniform(0.2, 2.0),
                                       rng.normal(0.0, 1.0), rng.normal(0.0, 1.0))
    return f, F, mask, mu, faces


def gpu(shape_xyz, f, F, mu, faces, bc, steps, precision="fp64", init="uniform", plan=None,
        rho=None):
    from paper_2603_22553_amd.lattice import Lattice
    with Lattice(shape_xyz, bc=tuple(NAMES[b] for b in bc), precision=precision,
                 n_regions=f.n_regions, max_records=steps + 1, mobility=mu is not None) as lat:
        if plan:
            lat.set_plan(*plan)
        lat.set_free_energy(F)
        lat.set_shift(f.delta)
        lat.set_regions(f.region)
        if mu is not None:
            lat.set_mobility(mu)
        for (axis, side), (Fg, rg, mre, mim) in faces.items():
            lat.set_reservoir(axis, side, Fg, rg, complex(mre, mim))
        if rho is not None:
            lat.init_state(rho=rho)
        else:
            lat.init_state(init)
        lat.run(steps)
        return lat.records(), lat.population(), lat.magnetization()


def check(tag, rec, rho, m, ref, R, precision):
    strict = precision == "fp64"
    U, Uo = rec[:, 2 * R:3 * R], ref.records[:, 2 * R:3 * R]
    eu = np.max(np.abs(U - Uo)) / np.max(np.abs(Uo))
    assert eu <= (1e-10 if strict else 1e-5), f"{tag}: uptake {eu}"
    G = rec[:, 0:2 * R:2].sum(1) + 1j * rec[:, 1:2 * R:2].sum(1)
    eg = rel_l2(G, ref.fid())
    assert eg <= (1e-10 if strict else 1e-3), f"{tag}: FID {eg}"
    for k in range(6):
        a, b = rec[:, 3 * R + k], ref.records[:, 3 * R + k]
        scale = max(np.max(np.abs(ref.records[:, 3 * R + 3 + k % 3])), 1.0)
        e = np.max(np.abs(a - b)) / scale
        assert e <= (1e-10 if strict else 1e-4), f"{tag}: moment {k} {e}"
    er = np.max(np.abs(rho.reshape(-1) - ref.rho)) / np.max(ref.rho)
    assert er <= (1e-10 if strict else 1e-5), f"{tag}: rho {er}"
    em = np.max(np.abs(m.reshape(-1) - (ref.re + 1j * ref.im))) / np.max(np.abs(ref.re + 1j * ref.im))
    assert em <= (1e-10 if strict else 1e-3), f"{tag}: m {em}"


CASES = [
    # shape, bc, mobility, obstacles
    ((70, 9, 23), (PER, PER, PER), False, 0.25),
    ((33, 40, 17), (CLO, PER, CLO), True, 0.15),
    ((70, 9, 23), (RES, PER, CLO), False, 0.1),
    ((33, 40, 17), (PER, RES, RES), True, 0.2),
    ((20, 12, 30), (RES, RES, RES), True, 0.1),
    ((1, 5, 3), (RES, PER, RES), False, 0.0),
    ((17, 1, 1), (CLO, RES, RES), True, 0.0),
]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[0])) + "-" +
                         "".join("PCR"[b] for b in c[1]) + ("-mob" if c[2] else ""))
def test_against_oracle(oracle, case, precision):
    shape, bc, mob, obst = case
    f, F, mask, mu, faces = scene(shape, seed=sum(shape) + 7 * bc[0] + 3 * bc[2], obstacles=obst,
                                  mobility=mob, bc=bc)
    steps = 150
    rec, rho, m = gpu(shape, f, F, mu, faces, bc, steps, precision)
    ref = oracle.run(F, f.delta, f.region, f.n_regions, steps, bc=bc, mobility=mu,
                     reservoir=faces or None)
    check(f"{shape} {bc} {precision}", rec, rho, m, ref, f.n_regions, precision)
    assert np.all(rho.reshape(-1)[mask.reshape(-1)] == 0.0)


@pytest.mark.parametrize("plan", [(64, 5), (32, 7), (16, 4)])
def test_every_tile_shape_and_z_chunk(oracle, plan):
    """Ghost halo slots of every tile width and ghost planes at chunked z-ends."""
    shape, bc = (50, 37, 29), (RES, RES, RES)
    f, F, mask, mu, faces = scene(shape, seed=91, obstacles=0.15, mobility=True, bc=bc)
    rec, rho, m = gpu(shape, f, F, mu, faces, bc, 60, plan=plan)
    ref = oracle.run(F, f.delta, f.region, f.n_regions, 60, bc=bc, mobility=mu, reservoir=faces)
    check(f"plan {plan}", rec, rho, m, ref, f.n_regions, "fp64")


def test_initial_states_hold_nothing_on_obstacles(oracle):
    """Uniform, Boltzmann (Eq. (2) over the accessible sites) and user starts are zero on
    the solid matrix; the Boltzmann populations equal the oracle's."""
    from paper_2603_22553_amd.lattice import Lattice
    f, F, mask, _, _ = scene((24, 16, 12), seed=93, obstacles=0.3)
    flat = mask.reshape(-1)
    with Lattice(f.shape_xyz, n_regions=2, max_records=2) as lat:
        lat.set_fields(f)
        lat.set_free_energy(F)
        lat.init_state("uniform")
        p = lat.population().reshape(-1)
        assert np.all(p[flat] == 0.0) and np.all(p[~flat] == 1.0)
        lat.init_state("boltzmann")
        p = lat.population().reshape(-1)
        eq = oracle.boltzmann(F).reshape(-1)
        assert np.max(np.abs(p - eq)) <= 1e-12 * eq.max()
        assert abs(p.sum() - (~flat).sum()) <= 1e-9
        lat.init_state(rho=np.full(f.n_sites, 2.0))
        p = lat.population().reshape(-1)
        assert np.all(p[flat] == 0.0) and np.all(p[~flat] == 2.0)
        assert np.all(lat.magnetization().reshape(-1)[flat] == 0.0)


def test_reservoir_equilibrium_closed_form(oracle):
    """Reservoir faces at one chemical potential fix the equilibrium to K exp(-F_i); the
    device equilibration reaches it from an empty lattice (and the run from it stays)."""
    from paper_2603_22553_amd.lattice import Lattice
    f = synth.random_fields((18, 10, 14), seed=95, F_scale=0.8)
    K = 1.7
    with Lattice(f.shape_xyz, bc=("reservoir", "periodic", "reservoir"), max_records=11) as lat:
        lat.set_fields(f)
        for axis in (0, 2):
            for side in (0, 1):
                Fg = 0.25 * side - 0.1 * axis
                lat.set_reservoir(axis, side, Fg, K * math.exp(-Fg))
        lat.init_state(rho=np.zeros(f.n_sites))
        steps, res = lat.equilibrate(200000, 1e-13, check_every=100)
        assert res <= 1e-13
        want = K * np.exp(-f.F)
        assert np.max(np.abs(lat.population() - want)) <= 1e-9 * want.max()
        lat.run(10)
        mass = lat.moments()[0]
        assert np.max(np.abs(mass / mass[0] - 1.0)) <= 1e-11


def test_reservoir_lattice_skips_the_conservation_alarm(oracle):
    """An empty reservoir drains the lattice: reads succeed although the total falls."""
    from paper_2603_22553_amd.lattice import Lattice
    f = synth.random_fields((12, 10, 8), seed=97)
    with Lattice(f.shape_xyz, bc=("reservoir", "periodic", "periodic"), max_records=101) as lat:
        lat.set_fields(f)
        lat.init_state()
        lat.run(100)
        mass = lat.moments()[0]
        assert mass[-1] < 0.99 * mass[0]
        lat.fid()
        lat.check()


def test_mixed_variant_batch_equals_solo():
    """Plain and extended lattices (mobility, reservoir faces) in one batch: each runs the
    kernel variant it runs alone and gives the same bits."""
    from paper_2603_22553_amd.lattice import Batch, Lattice
    specs = [((40, 24, 19), (PER, PER, CLO), False, 100), ((40, 24, 19), (RES, PER, CLO), True, 101),
             ((17, 33, 12), (PER, RES, RES), False, 102), ((64, 8, 9), (CLO, CLO, RES), True, 103),
             ((33, 20, 11), (CLO, PER, PER), True, 104)]

    def make(shape, bc, mob, seed):
        f, F, mask, mu, faces = scene(shape, seed=seed, obstacles=0.1, mobility=mob, bc=bc)
        lat = Lattice(shape, bc=tuple(NAMES[b] for b in bc), n_regions=2, max_records=81,
                      mobility=mob)
        lat.set_fields(f)
        lat.set_free_energy(F)
        if mob:
            lat.set_mobility(mu)
        for (axis, side), (Fg, rg, mre, mim) in faces.items():
            lat.set_reservoir(axis, side, Fg, rg, complex(mre, mim))
        lat.init_state()
        return lat

    solo = []
    for s in specs:
        with make(*s) as lat:
            lat.run(80)
            solo.append(lat.records())
    lats = [make(*s) for s in specs]
    b = Batch(lats)
    b.run(80)
    b.close()
    for lat, ref in zip(lats, solo):
        assert np.array_equal(lat.records(), ref)
        lat.close()


def test_errors():
    from paper_2603_22553_amd import _native as N
    from paper_2603_22553_amd.lattice import Lattice
    f = synth.random_fields((8, 8, 8), seed=99)
    with Lattice((8, 8, 8), max_records=2) as lat:
        with pytest.raises(N.LpcError) as e:
            lat.set_mobility(np.ones(512))
        assert e.value.status == N.LPC_ERR_STATE
        with pytest.raises(N.LpcError) as e:
            lat.set_reservoir(0, 0, 0.0, 1.0)
        assert e.value.status == N.LPC_ERR_STATE
        for bad, code in ((-INF, N.LPC_ERR_NONFINITE), (np.nan, N.LPC_ERR_NONFINITE),
                          (2e30, N.LPC_ERR_ARG), (1500.0, N.LPC_ERR_ARG)):
            F = f.F.copy()
            F[1, 2, 3] = bad
            with pytest.raises(N.LpcError) as e:
                lat.set_free_energy(F)
            assert e.value.status == code
    with Lattice((8, 8, 8), bc=("periodic", "reservoir", "closed"), mobility=True,
                 max_records=2) as lat:
        for mu, code in ((1.5, N.LPC_ERR_ARG), (-0.1, N.LPC_ERR_ARG),
                         (np.nan, N.LPC_ERR_NONFINITE)):
            a = np.ones(512)
            a[7] = mu
            with pytest.raises(N.LpcError) as e:
                lat.set_mobility(a)
            assert e.value.status == code
        for args, code in (((3, 0), N.LPC_ERR_ARG), ((1, 2), N.LPC_ERR_ARG),
                           ((2, 0), N.LPC_ERR_STATE)):
            with pytest.raises(N.LpcError) as e:
                lat.set_reservoir(*args, 0.0, 1.0)
            assert e.value.status == code
        with pytest.raises(N.LpcError) as e:
            lat.set_reservoir(1, 0, 0.0, -1.0)
        assert e.value.status == N.LPC_ERR_ARG
        with pytest.raises(N.LpcError) as e:
            lat.set_reservoir(1, 1, INF, 1.0)
        assert e.value.status == N.LPC_ERR_NONFINITE


def test_extended_checkpoint_restart_bitwise():
    """An extended lattice (mobility, reservoir faces, obstacles) restarts bit for bit from a
    checkpoint once its fields and reservoir values are set again (fields are inputs, not
    state)."""
    from paper_2603_22553_amd.lattice import Lattice
    shape, bc = (30, 17, 21), (RES, PER, RES)
    f, F, mask, mu, faces = scene(shape, seed=131, obstacles=0.15, mobility=True, bc=bc)

    def make():
        lat = Lattice(shape, bc=tuple(NAMES[b] for b in bc), n_regions=2, max_records=101,
                      mobility=True)
        lat.set_fields(f)
        lat.set_free_energy(F)
        lat.set_mobility(mu)
        for (axis, side), (Fg, rg, mre, mim) in faces.items():
            lat.set_reservoir(axis, side, Fg, rg, complex(mre, mim))
        return lat

    with make() as full:
        full.init_state()
        full.run(100)
        want = full.records(), full.population()
    with make() as a:
        a.init_state()
        a.run(40)
        blob = a.save_state()
    with make() as b:
        b.load_state(blob)
        b.run(60)
        assert np.array_equal(b.records(), want[0])
        assert np.array_equal(b.population(), want[1])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_porous_full_size(oracle, precision):
    """The porous 256^3 workload (a quarter of the carbon solid, pore-width mobility, bulk
    reservoir faces in x) at full size in the benchmark's launch configuration, over a short
    prefix the oracle finishes in seconds."""
    f, mu = synth.porous_particle()
    faces = {(0, 0): (0.0, 1.0, 1.0, 0.0), (0, 1): (0.0, 1.0, 1.0, 0.0)}
    steps = 3
    bc = (RES, PER, PER)
    rec, rho, m = gpu(f.shape_xyz, f, f.F, mu, faces, bc, steps, precision, init="boltzmann")
    ref = oracle.run(f.F, f.delta, f.region, f.n_regions, steps, bc=bc, mobility=mu,
                     reservoir=faces, init="boltzmann")
    check(f"porous 256^3 {precision}", rec, rho, m, ref, f.n_regions, precision)
