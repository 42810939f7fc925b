"""Equilibration phase and the velocity autocorrelation on the GPU path, against the oracle.

The equilibration (section 3.2) steps the populations alone until their largest one-step
change, relative to the largest population, is below a threshold; the propagation then
restarts from those populations. The autocorrelation of Eq. (4) is read back from the
recorded mean-square displacement of a run started at equilibrium.
"""
import numpy as np
import pytest

from conftest import rel_l2
from oracle import brute
from paper_2603_22553_amd import synth

pytestmark = pytest.mark.gpu

PER, CLO = 0, 1
P0 = 1.0 / 7.0


def lattice(f, bc=(PER, PER, PER), **kw):
    from paper_2603_22553_amd.lattice import Lattice
    bcs = tuple("periodic" if b == PER else "closed" for b in bc)
    lat = Lattice(f.shape_xyz, bc=bcs, n_regions=f.n_regions, **kw)
    lat.set_fields(f)
    return lat


@pytest.mark.parametrize("bc", [(PER, PER, PER), (CLO, PER, CLO)])
def test_equilibrate_fp64_matches_oracle(oracle, bc):
    """Same stopping step as the oracle (within one step: the crossing of the threshold
    may move by one under a different rounding order) and the same populations."""
    f = synth.random_fields((21, 10, 9), seed=51, F_scale=1.0)
    tol = 1e-11
    rho_o, steps_o, _ = oracle.equilibrate(f.F, 50000, tol, bc=bc)
    with lattice(f, bc, max_records=101) as lat:
        lat.init_state("uniform")
        steps, res = lat.equilibrate(50000, tol, check_every=1)
        assert abs(steps - steps_o) <= 1 and res <= tol
        assert lat.steps_done == 0
        rho = lat.population()
        assert np.max(np.abs(rho - rho_o)) <= 1e-10 * rho_o.max()
        # distance to the fixed point is about the last change over the spectral gap
        eq = oracle.boltzmann(f.F)
        assert np.max(np.abs(rho - eq)) <= 5e-8 * eq.max()
        # the propagation restarts from the equilibrated populations with m = rho
        m = lat.magnetization()
        assert np.array_equal(m.real, rho) and np.all(m.imag == 0.0)
        lat.run(100)
        rec = lat.records()
    ref = oracle.run(f.F, f.delta, f.region, f.n_regions, 100, bc=bc, init=rho_o)
    G = rec[:, 0] + 1j * rec[:, 1]
    assert rel_l2(G, ref.fid()) <= 1e-10
    assert np.max(np.abs(rec[:, 6:9] - ref.s2())) <= 1e-10 * np.max(ref.s2())


def test_equilibrate_check_interval_and_cap(oracle):
    """Checks every k steps stop at the first multiple of k past the oracle's step; the
    cap stops the phase with the last change reported; a second call from equilibrium
    stops at its first check."""
    f = synth.random_fields((16, 12, 8), seed=53)
    tol = 1e-10
    _, steps_o, _ = oracle.equilibrate(f.F, 50000, tol)
    with lattice(f, max_records=11) as lat:
        lat.init_state("uniform")
        steps, res = lat.equilibrate(50000, tol, check_every=25)
        assert steps % 25 == 0 and steps_o - 1 <= steps <= steps_o + 25
        steps, res = lat.equilibrate(1000, tol, check_every=10)
        assert steps == 10 and res <= tol
    with lattice(f, max_records=11) as lat:
        lat.init_state("uniform")
        steps, res = lat.equilibrate(30, 0.0, check_every=7)
        assert steps == 30 and res > 0.0
        _, steps_o, res_o = oracle.equilibrate(f.F, 30, 0.0)
        assert abs(res - res_o) <= 1e-9 * res_o


def test_equilibrate_mixed_precision(oracle):
    """The mixed path keeps populations in FP64 and rounds hop probabilities to FP32, so its
    fixed point sits within FP32 rounding of Boltzmann."""
    f = synth.random_fields((40, 24, 19), seed=55, n_regions=2)
    with lattice(f, precision="mixed", max_records=2) as lat:
        lat.init_state("uniform")
        steps, res = lat.equilibrate(50000, 1e-10, check_every=50)
        assert res <= 1e-10 and 0 < steps < 50000
        rho = lat.population()
    eq = oracle.boltzmann(f.F)
    assert abs(rho.sum() - f.n_sites) <= 1e-12 * f.n_sites
    assert np.max(np.abs(rho - eq)) <= 1e-5 * eq.max()


def test_equilibrate_errors():
    from paper_2603_22553_amd import _native as N
    f = synth.random_fields((8, 8, 8), seed=57)
    with lattice(f, max_records=2) as lat:
        with pytest.raises(N.LpcError) as e:
            lat.equilibrate(10, 1e-10)
        assert e.value.status == N.LPC_ERR_STATE
        lat.init_state()
        for args in ((-1, 1e-10, 1), (10, -1.0, 1), (10, float("nan"), 1), (10, 1e-10, 0)):
            with pytest.raises(N.LpcError) as e:
                lat.equilibrate(*args)
            assert e.value.status == N.LPC_ERR_ARG
        with pytest.raises(N.LpcError) as e:
            lat.vacf()                       # fewer than two steps recorded
        assert e.value.status == N.LPC_ERR_STATE
    with lattice(f, max_records=5, track=("fid",)) as lat:
        lat.init_state()
        lat.run(4)
        with pytest.raises(N.LpcError) as e:
            lat.vacf()
        assert e.value.status == N.LPC_ERR_STATE


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 2e-3)])
def test_vacf_against_dense(oracle, precision, tol):
    """Eq. (4): the autocorrelation read from the GPU's MSD equals the dense C(tau) computed
    from the one-step matrices, on a 4^3 lattice with a closed axis."""
    f = synth.random_fields((4, 4, 4), seed=59, F_scale=1.2)
    bc = (CLO, PER, PER)
    t = 40
    with lattice(f, bc, precision=precision, max_records=t + 1) as lat:
        lat.init_state("boltzmann")
        lat.run(t)
        C = lat.vacf()
        D = lat.kohn_diffusion()
        msd = lat.records()[:, 6:9] / lat.records()[:, 2:3]
    rho_eq = oracle.boltzmann(f.F).reshape(-1)
    for a in range(3):
        T0, T1, T2 = brute.matrices((4, 4, 4), bc, f.F, P0, axis=a)
        want = brute.vacf(T0, T1, T2, rho_eq, t) / rho_eq.sum()
        assert np.max(np.abs(C[:, a] - want)) <= tol * want[0], a
    # the truncated Kohn sum telescopes to half the last MSD increment
    a2, dt = 0.5e-9 ** 2, 5e-6
    assert np.allclose(D, a2 * (msd[t] - msd[t - 1]) / (2 * dt), rtol=1e-9, atol=0)


def test_kohn_d_after_equilibration(oracle):
    """Equilibrate from a uniform start, then propagate: the Kohn D at a long lag agrees
    with the oracle's run from its own equilibrated populations (both stop within one step
    of each other, so their starting populations differ by about the threshold)."""
    f = synth.random_fields((24, 20, 16), seed=61)
    t = 300
    rho_o, _, _ = oracle.equilibrate(f.F, 50000, 1e-12)
    ref = oracle.run(f.F, f.delta, f.region, 1, t, init=rho_o)
    msd_o = ref.msd()
    with lattice(f, max_records=t + 1) as lat:
        lat.init_state("uniform")
        lat.equilibrate(50000, 1e-12, check_every=1)
        lat.run(t)
        C = lat.vacf()
        D = lat.kohn_diffusion()
    c_o = np.vstack([msd_o[1] - msd_o[0], 0.5 * (msd_o[2:] - 2 * msd_o[1:-1] + msd_o[:-2])])
    assert np.max(np.abs(C - c_o)) <= 1e-8 * np.max(np.abs(c_o))
    D_o = 0.5e-9 ** 2 * (msd_o[t] - msd_o[t - 1]) / (2 * 5e-6)
    assert np.allclose(D, D_o, rtol=1e-8, atol=0)
