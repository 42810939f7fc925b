"""The velocity autocorrelation field (LPC_TRACK_VACF): each particle carries its first
displacement in a tag field, so that Eq. (4)'s C(tau) = <dx_1 dx_{1+tau}> is recorded every
step without differencing the mean-square displacement. Against the dense one-step matrices,
the oracle's own tag recursion, and the Einstein sum of the displacement moments."""
import numpy as np
import pytest

from oracle import brute
from paper_2603_22553_amd import _native as N
from paper_2603_22553_amd import synth

pytestmark = pytest.mark.gpu

PER, CLO, RES = 0, 1, 2
NAMES = ("periodic", "closed", "reservoir")
P0 = 1.0 / 7.0
TRACK = ("fid", "msd", "vacf")
# FP64 at rounding; the mixed path moves the tags in float (2^-24 per step)
TOL = {"fp64": 1e-10, "mixed": 1e-5}


def lattice(f, bc, precision, steps, **kw):
    from paper_2603_22553_amd.lattice import Lattice
    return Lattice(f.shape_xyz, bc=tuple(NAMES[b] for b in bc), precision=precision,
                   track=TRACK, n_regions=f.n_regions, max_records=steps + 1, **kw)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_vacf_field_against_dense(precision):
    f = synth.random_fields((4, 4, 4), seed=59, F_scale=1.2)
    bc = (CLO, PER, PER)
    t = 60
    with lattice(f, bc, precision, t) as lat:
        lat.set_fields(f)
        lat.init_state("boltzmann")
        lat.run(t)
        C = lat.vacf()
        rec = lat.records()
    assert np.all(rec[0, -3:] == 0.0)
    from oracle import oracle
    rho_eq = oracle.boltzmann(f.F).reshape(-1)
    for a in range(3):
        T0, T1, T2 = brute.matrices((4, 4, 4), bc, f.F.reshape(-1), P0, axis=a)
        want = brute.vacf(T0, T1, T2, rho_eq, t) / rho_eq.sum()
        assert np.max(np.abs(C[:, a] - want)) <= TOL[precision] * want[0], a


CASES = [
    # shape, bc, F scale, obstacles, mobility, start
    ((24, 20, 16), (PER, PER, PER), 1.0, False, False, "boltzmann"),
    ((37, 11, 9), (CLO, PER, CLO), 1.5, False, False, "uniform"),
    ((20, 18, 15), (PER, CLO, PER), 1.0, True, True, "boltzmann"),
    ((16, 12, 10), (RES, PER, PER), 1.0, True, False, "boltzmann"),
    ((12, 10, 9), (PER, RES, RES), 0.8, False, True, "uniform"),
]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[0])) + "-" +
                         "".join("PCR"[b] for b in c[1]))
def test_vacf_field_against_oracle(oracle, precision, case):
    """The tag recursion against the oracle's, with obstacles, link mobility and reservoir
    faces (a particle that enters from a reservoir carries no tag), from equilibrium and from
    a uniform start (the tags need no stationary start)."""
    shape, bc, Fs, obst, mob, start = case
    f = synth.random_fields(shape, seed=sum(shape) + bc[0], F_scale=Fs)
    rng = np.random.default_rng(sum(shape))
    if obst:
        f.F[rng.random(f.F.shape) < 0.1] = np.inf
    mu = rng.uniform(0.2, 1.0, size=f.F.shape) if mob else None
    reservoir = {(a, s): (0.3, 1.0, 1.0, 0.0) for a in range(3) if bc[a] == RES for s in (0, 1)}
    t = 150
    with lattice(f, bc, precision, t, mobility=mob) as lat:
        lat.set_fields(f)
        if mob:
            lat.set_mobility(mu)
        for (a, s), v in reservoir.items():
            lat.set_reservoir(a, s, v[0], v[1], complex(v[2], v[3]))
        lat.init_state(start)
        lat.run(t)
        C = lat.vacf()
    rho0 = oracle.boltzmann(f.F) if start == "boltzmann" else np.where(np.isinf(f.F), 0.0, 1.0)
    want = oracle.vacf(f.F, t, bc=bc, rho=rho0, mobility=mu, reservoir=reservoir or None)
    assert np.max(np.abs(C - want)) <= TOL[precision] * np.max(np.abs(want[0]))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_vacf_field_einstein_at_long_lags(precision):
    """From equilibrium, the moments' MSD equals the Einstein sum of the tag field's C at
    every lag up to 1500 steps: two recursions on the device, agreeing to rounding (the
    mixed path: both in float storage)."""
    f = synth.particle(24, 8, 2.0, (0.7, 2.0), seed=9)
    t = 1500
    with lattice(f, (PER, PER, CLO), precision, t) as lat:
        lat.set_fields(f)
        lat.init_state("boltzmann")
        lat.run(t)
        C = lat.vacf()
        _, msd, _ = lat.moments()
        D_kohn = lat.kohn_diffusion()
        D_slope, _ = lat.diffusion()
    tol = 1e-9 if precision == "fp64" else 2e-4
    for a in range(3):
        for tt in (1, 10, 100, 1000, t):
            want = brute.msd_from_vacf(C[:, a], tt)
            assert abs(msd[tt, a] - want) <= tol * msd[tt, a], (a, tt)
    # Eq. (4) at the longest lag against the MSD slope of the second half (closed z: the
    # autocorrelation has decayed long before)
    np.testing.assert_allclose(D_kohn[:2], D_slope[:2], rtol=2e-3)


def test_vacf_batch_and_checkpoint_bitwise():
    """The tagging step runs alone before a batch joins: a batched lattice ends on the bits of
    a solo run, and a run continued from a checkpoint on those of an unbroken run."""
    from paper_2603_22553_amd.lattice import Batch
    f = synth.random_fields((30, 22, 14), seed=71, n_regions=2)
    g = synth.random_fields((17, 13, 11), seed=72, n_regions=2)

    def make(x):
        lat = lattice(x, (PER, CLO, PER), "mixed", 400)
        lat.set_fields(x)
        lat.init_state("boltzmann")
        return lat

    with make(f) as a, make(g) as b, make(f) as solo, make(f) as split:
        with Batch([a, b]) as bt:
            bt.run([300, 120])
        solo.run(300)
        assert np.array_equal(a.records(), solo.records())
        assert np.array_equal(a.population(), solo.population())
        split.run(5)
        blob = split.save_state()
        split.init_state("uniform")
        split.load_state(blob)
        split.run(295)
        assert np.array_equal(split.records(), solo.records())


def test_vacf_errors():
    from paper_2603_22553_amd.lattice import Lattice
    with pytest.raises(N.LpcError) as e:
        Lattice((8, 8, 8), track=("fid", "vacf"), max_records=3)
    assert e.value.status == N.LPC_ERR_ARG
    with Lattice((40, 40, 40), track=TRACK, max_records=3) as lat:
        with pytest.raises(N.LpcError) as e:
            lat.set_plan(2, 0)
        assert e.value.status == N.LPC_ERR_ARG
        assert lat.K == 3 + 6 + 3
