"""Pins of the CPU FP64 oracle against facts the paper and the mathematics fix.

Each test names the passage it follows. None of them retypes the oracle's update: they
compare it with hand-derived values, closed forms, invariants and an independent dense
brute force (oracle/brute.py).
"""
import math

import numpy as np
import pytest

from conftest import load_golden, parse_value, rel_l2
from oracle import brute
from paper_2603_22553_amd import synth

P0 = 1.0 / 7.0
DT = 5e-6
NU0 = 400e6
PER, CLO = 0, 1


def _flat(a):
    return np.asarray(a, dtype=np.float64).reshape(-1)


# --------------------------------------------------------------------- hand-derived cases

@pytest.mark.parametrize("case", load_golden("hand_cases.json")["cases"], ids=lambda c: c["name"])
def test_hand_cases(oracle, case):
    """Tiny lattices stepped by hand (Eqs. (1), (5), (7), (13); moment propagation; the
    Dirichlet ghost sites of section 3.2)."""
    nx, ny, nz = case["shape_xyz"]
    bc = tuple({"periodic": PER, "closed": CLO, "reservoir": 2}[b] for b in case["bc"])
    reservoir = {tuple(int(v) for v in k.split(",")): tuple(parse_value(x) for x in vals)
                 for k, vals in case.get("reservoir", {}).items()} or None
    mobility = (np.array([parse_value(v) for v in case["mobility"]]).reshape(nz, ny, nx)
                if "mobility" in case else None)
    init = case.get("init", "uniform")
    if not isinstance(init, str):
        init = np.array([parse_value(v) for v in init]).reshape(nz, ny, nx)
    F = np.array([parse_value(v) for v in case["F"]]).reshape(nz, ny, nx)
    delta = np.array([parse_value(v) for v in case["delta_ppm"]]).reshape(nz, ny, nx)
    region = np.array(case["region"], dtype=np.uint8).reshape(nz, ny, nx)
    R = case["n_regions"]
    last = max(s["n"] for s in case["steps"])
    for step in case["steps"]:
        res = oracle.run(F, delta, region, R, step["n"], bc=bc, p0=parse_value(case["p0"]),
                         dt=case["dt"], nu0=case["nu0"], init=init, reservoir=reservoir,
                         mobility=mobility)
        want = {k: np.array([parse_value(v) for v in step[k]]) for k in
                ("rho", "m_re", "m_im", "S1", "S2")}
        np.testing.assert_allclose(res.rho, want["rho"], rtol=0, atol=1e-15)
        np.testing.assert_allclose(res.re, want["m_re"], rtol=0, atol=1e-15)
        np.testing.assert_allclose(res.im, want["m_im"], rtol=0, atol=1e-15)
        np.testing.assert_allclose(res.s1()[-1], want["S1"], rtol=0, atol=1e-15)
        np.testing.assert_allclose(res.s2()[-1], want["S2"], rtol=0, atol=1e-15)
        # per-region records are the sums of the final state over the region's sites
        for r in range(R):
            sel = case["region"]
            G = sum(complex(want["m_re"][i], want["m_im"][i]) for i in range(len(sel)) if sel[i] == r)
            U = sum(want["rho"][i] for i in range(len(sel)) if sel[i] == r)
            assert abs(res.fid(r)[-1] - G) < 1e-15
            assert abs(res.uptake()[-1, r] - U) < 1e-15
    assert last >= 1


# --------------------------------------------------------------------- P1 conservation

@pytest.mark.parametrize("bc", [(PER, PER, PER), (CLO, PER, PER), (CLO, CLO, CLO)])
def test_mass_conservation(oracle, bc):
    """Columns of the transition sum to one (stay + all moves out), so mass is exact (sec. 2.1)."""
    f = synth.random_fields((7, 6, 5), seed=11, F_scale=2.0, n_regions=3)
    res = oracle.run(f.F, f.delta, f.region, 3, 500, bc=bc)
    m = res.mass()
    assert np.max(np.abs(m / m[0] - 1.0)) <= 1e-12


def test_mass_conservation_single_particle(oracle):
    """32^3 particle (generator of the small single-particle workload), 5000 steps."""
    f = synth.single_particle_small()
    res = oracle.run(f.F, f.delta, f.region, 2, 5000, moments=False)
    m = res.mass()
    assert np.max(np.abs(m / m[0] - 1.0)) <= 1e-12


# --------------------------------------------------------------------- P2 detailed balance

@pytest.mark.parametrize("bc", [(PER, PER, PER), (CLO, PER, CLO)])
def test_boltzmann_is_stationary(oracle, bc):
    """Eq. (2): populations proportional to exp(-F) are unchanged by a step (detailed balance)."""
    f = synth.random_fields((6, 5, 4), seed=3, F_scale=1.5)
    rho_eq = oracle.boltzmann(f.F)
    res = oracle.run(f.F, f.delta, f.region, 1, 1, bc=bc, init="boltzmann")
    assert np.max(np.abs(res.rho / _flat(rho_eq) - 1.0)) <= 1e-14


def test_uniform_start_converges_to_boltzmann(oracle):
    """A uniform start relaxes to Eq. (2) with <rho> = 1."""
    f = synth.random_fields((4, 4, 4), seed=5, F_scale=1.0)
    res = oracle.run(f.F, f.delta, f.region, 1, 3000, moments=False)
    rho_eq = _flat(oracle.boltzmann(f.F))
    assert np.max(np.abs(res.rho / rho_eq - 1.0)) <= 1e-10


# --------------------------------------------------------------------- P3 single line

def test_uniform_shift_single_line(oracle):
    """With one shift everywhere, G(n) = exp(i n theta) G(0) whatever F is (Eqs. (8), (13))."""
    f = synth.random_fields((6, 5, 7), seed=8, F_scale=1.0, n_regions=2)
    d_ppm = -3.7
    delta = np.full_like(f.F, d_ppm)
    n = 400
    res = oracle.run(f.F, delta, f.region, 2, n)
    theta = 2 * math.pi * d_ppm * 1e-6 * NU0 * DT
    G = res.fid()
    want = G[0] * np.exp(1j * theta * np.arange(n + 1))
    assert np.max(np.abs(G - want)) / abs(G[0]) <= 1e-12


def test_uniform_shift_spectrum_peak(oracle):
    """The spectrum (Eq. (9)) of a single line peaks at its shift: sign and 2 pi of Eq. (11)."""
    f = synth.random_fields((5, 5, 5), seed=9, F_scale=1.0)
    for d_ppm in (-6.3, -0.8, 2.45):
        delta = np.full_like(f.F, d_ppm)
        res = oracle.run(f.F, delta, f.region, 1, 2000, moments=False)
        assert abs(oracle.peak_ppm(res.fid(), DT, NU0) - d_ppm) <= 0.01


# --------------------------------------------------------------------- P4 free lattice

def test_free_lattice_msd(oracle):
    """F = 0, periodic: iid moves, so MSD_a(n) = 2 p0 n and D = a^2 / (7 dt) (Eqs. (6)-(7))."""
    shape = (6, 5, 4)
    F = np.zeros(shape[::-1])
    res = oracle.run(F, np.zeros_like(F), np.zeros(F.shape, np.uint8), 1, 100)
    n = np.arange(101)
    for a in range(3):
        np.testing.assert_allclose(res.msd()[:, a], 2 * P0 * n, rtol=1e-12, atol=1e-13)
        assert np.max(np.abs(res.drift()[:, a])) <= 1e-13
    D, slope = oracle.diffusion(res.msd(), DT, 0.5e-9)
    np.testing.assert_allclose(D, (0.5e-9) ** 2 / (7 * DT), rtol=1e-12)
    np.testing.assert_allclose(oracle.diffusion_ratio(res.msd(), P0), 1.0, rtol=1e-12)


def test_free_lattice_msd_alpha(oracle):
    """Eq. (7) for another alpha = 6 p0: MSD slope 2 p0 per step along each axis."""
    F = np.zeros((4, 4, 4))
    p0 = 0.05
    res = oracle.run(F, np.zeros_like(F), np.zeros(F.shape, np.uint8), 1, 50, p0=p0)
    np.testing.assert_allclose(res.msd()[-1], [2 * p0 * 50] * 3, rtol=1e-12)


# --------------------------------------------------------------------- P5 Eq. (5)

def test_one_step_msd_eq5(oracle):
    """Eq. (5): after one step from equilibrium, <dx^2> = sum_i rho_i sum_j p(i->j) a_x^2 / sum rho."""
    f = synth.random_fields((5, 4, 6), seed=21, F_scale=1.3)
    nx, ny, nz = f.shape_xyz
    res = oracle.run(f.F, f.delta, f.region, 1, 1, init="boltzmann")
    rho = oracle.boltzmann(f.F)
    F = f.F
    # forward sum over sites i and their moves i -> j along each axis (periodic)
    want = np.zeros(3)
    for a, ax in enumerate((2, 1, 0)):
        for s in (+1, -1):
            Fj = np.roll(F, -s, axis=ax)
            p = P0 * np.minimum(1.0, np.exp(-(Fj - F)))
            want[a] += np.sum(rho * p)
    want /= rho.sum()
    np.testing.assert_allclose(res.msd()[1], want, rtol=1e-14)


# --------------------------------------------------------------------- P6 dense brute force

@pytest.mark.parametrize("bc", [(PER, PER, PER), (CLO, PER, CLO), (PER, CLO, CLO)])
def test_dense_brute_force(oracle, bc):
    """4^3 lattice: oracle FID and moments against dense matrices built link by link."""
    f = synth.random_fields((4, 4, 4), seed=17, F_scale=1.2, delta_scale=8.0)
    n = 300
    res = oracle.run(f.F, f.delta, f.region, 1, n, bc=bc)
    theta = brute.phases(f.delta, DT, NU0)
    T0, _, _ = brute.matrices((4, 4, 4), bc, f.F, P0, axis=0)
    G = brute.fid(T0, theta, np.ones(64), n)
    assert rel_l2(res.fid(), G) <= 1e-12
    for a in range(3):
        T0a, T1a, T2a = brute.matrices((4, 4, 4), bc, f.F, P0, axis=a)
        mom = brute.moments(T0a, T1a, T2a, np.ones(64), n)
        np.testing.assert_allclose(res.mass(), mom[:, 0], rtol=1e-13)
        np.testing.assert_allclose(res.s1()[:, a], mom[:, 1], rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(res.s2()[:, a], mom[:, 2], rtol=1e-12)


def test_dense_matrix_power_long(oracle):
    """G(20000) of the 4^3 lattice against numpy's repeated-squaring matrix power."""
    f = synth.random_fields((4, 4, 4), seed=19, F_scale=1.0, delta_scale=6.0)
    n = 20000
    res = oracle.run(f.F, f.delta, f.region, 1, n, moments=False)
    theta = brute.phases(f.delta, DT, NU0)
    T0, _, _ = brute.matrices((4, 4, 4), (PER, PER, PER), f.F, P0)
    for k in (1, 777, n):
        g = brute.fid_power(T0, theta, np.ones(64), k).sum()
        assert abs(res.fid()[k] - g) <= 1e-12 * abs(res.fid()[0])


def test_odd_sides_brute_force(oracle):
    """3x5x2 lattice (odd and size-2 periodic axes: two distinct links join the same pair)."""
    f = synth.random_fields((3, 5, 2), seed=23, F_scale=1.0, delta_scale=5.0)
    n = 200
    res = oracle.run(f.F, f.delta, f.region, 1, n)
    theta = brute.phases(f.delta, DT, NU0)
    for a in range(3):
        T0, T1, T2 = brute.matrices((3, 5, 2), (PER, PER, PER), f.F, P0, axis=a)
        if a == 0:
            assert rel_l2(res.fid(), brute.fid(T0, theta, np.ones(30), n)) <= 1e-12
        mom = brute.moments(T0, T1, T2, np.ones(30), n)
        np.testing.assert_allclose(res.s2()[:, a], mom[:, 2], rtol=1e-12)


# --------------------------------------------------------------------- P7 Kohn / VACF

def test_einstein_equals_kohn(oracle):
    """Eq. (4): from equilibrium, the moment-propagated MSD equals the Einstein sum of the
    discrete velocity autocorrelation (computed independently from dense matrices)."""
    f = synth.random_fields((4, 4, 4), seed=29, F_scale=1.5)
    t = 400
    res = oracle.run(f.F, f.delta, f.region, 1, t, init="boltzmann")
    rho_eq = _flat(oracle.boltzmann(f.F))
    T0, T1, T2 = brute.matrices((4, 4, 4), (PER, PER, PER), f.F, P0, axis=0)
    C = brute.vacf(T0, T1, T2, rho_eq, t)
    for tt in (1, 2, 10, 133, t):
        want = brute.msd_from_vacf(C, tt) / rho_eq.sum()
        assert abs(res.msd()[tt, 0] - want) <= 1e-12 * want


def test_vacf_from_msd_second_difference(oracle):
    """Eq. (4): the second difference of the moment-propagated MSD from equilibrium gives
    back the dense velocity autocorrelation (C(0) = MSD(1), C(tau) = half the second
    difference); summed, it is the Kohn D of Eq. (4) truncated at the last lag."""
    f = synth.random_fields((4, 4, 4), seed=37, F_scale=1.2)
    t = 60
    res = oracle.run(f.F, f.delta, f.region, 1, t, init="boltzmann", bc=(CLO, PER, PER))
    rho_eq = _flat(oracle.boltzmann(f.F))
    for a in range(3):
        T0, T1, T2 = brute.matrices((4, 4, 4), (CLO, PER, PER), f.F, P0, axis=a)
        C = brute.vacf(T0, T1, T2, rho_eq, t) / rho_eq.sum()
        msd = res.msd()[:, a]
        got = np.concatenate([[msd[1] - msd[0]], 0.5 * (msd[2:] - 2 * msd[1:-1] + msd[:-2])])
        assert np.max(np.abs(got - C)) <= 1e-12 * C[0]


def test_tag_vacf_equals_dense(oracle):
    """Eq. (4) by a tag field (each particle carries its first displacement, propagated like
    a population) against the dense C(tau) = 1^T T1 T0^(tau-1) T1 rho of the one-step
    matrices, on every axis, with a closed axis, obstacles and link mobility."""
    f = synth.random_fields((4, 4, 4), seed=43, F_scale=1.3)
    F = f.F.copy()
    F[0, 1, 2] = F[3, 2, 0] = np.inf
    mu = np.random.default_rng(44).uniform(0.3, 1.0, size=F.shape)
    t = 50
    bc = (CLO, PER, PER)
    got = oracle.vacf(F, t, bc=bc, mobility=mu)
    rho_eq = _flat(oracle.boltzmann(F))
    for a in range(3):
        T0, T1, T2 = brute.matrices((4, 4, 4), bc, _flat(F), P0, axis=a, mobility=_flat(mu))
        want = brute.vacf(T0, T1, T2, rho_eq, t) / rho_eq.sum()
        assert np.max(np.abs(got[:, a] - want)) <= 1e-12 * want[0], a


def test_tag_vacf_einstein_identity(oracle):
    """From equilibrium, the displacement moments (propagated by the sweep's own recursion)
    and the tag-field autocorrelation (a separate recursion) satisfy the Einstein sum:
    MSD(t) = t C(0) + 2 sum_{tau<t} (t - tau) C(tau), at every t checked."""
    f = synth.random_fields((5, 4, 6), seed=47, F_scale=1.0)
    t = 120
    bc = (PER, CLO, PER)
    res = oracle.run(f.F, f.delta, f.region, 1, t, init="boltzmann", bc=bc)
    C = oracle.vacf(f.F, t, bc=bc)
    for a in range(3):
        for tt in (1, 2, 7, 60, t):
            want = brute.msd_from_vacf(C[:, a], tt)
            assert abs(res.msd()[tt, a] - want) <= 1e-12 * want, (a, tt)


def test_tag_vacf_free_lattice(oracle):
    """F = 0, periodic: steps are independent, C(0) = 2 p0 (Eq. (7)) and C(tau >= 1) = 0; with
    a closed axis the walls reflect: C(0) = 2 p0 (1 - 1/n) and the first lag is negative."""
    F = np.zeros((6, 5, 7))
    C = oracle.vacf(F, 20)
    np.testing.assert_allclose(C[0], 2 * P0, rtol=1e-14)
    assert np.max(np.abs(C[1:])) <= 1e-16
    C = oracle.vacf(F, 20, bc=(CLO, PER, PER))
    assert abs(C[0, 0] - 2 * P0 * (1 - 1 / 7)) <= 1e-14
    assert C[1, 0] < 0 and np.max(np.abs(C[1:, 1:])) <= 1e-16


# --------------------------------------------------------------------- P8a equilibration

@pytest.mark.parametrize("bc", [(PER, PER, PER), (CLO, PER, CLO)])
def test_equilibration_reaches_stationary_vector(oracle, bc):
    """Equilibration phase (section 3.2): population steps alone until their one-step change
    is below the threshold. The result is the eigenvector of the dense one-step matrix for
    eigenvalue 1 (found by scipy's null space, not by stepping) and, by detailed balance,
    the Boltzmann populations of Eq. (2)."""
    import scipy.linalg
    f = synth.random_fields((5, 4, 3), seed=41, F_scale=1.0)
    rho, steps, res = oracle.equilibrate(f.F, 100000, 1e-13, bc=bc)
    assert 0 < steps < 100000 and res <= 1e-13
    assert abs(rho.sum() - f.n_sites) <= 1e-12 * f.n_sites           # mass kept
    T0, _, _ = brute.matrices((5, 4, 3), bc, f.F, P0)
    v = scipy.linalg.null_space(T0 - np.eye(f.n_sites))[:, 0]
    v = v * f.n_sites / v.sum()
    assert np.max(np.abs(_flat(rho) - v)) <= 1e-9 * v.max()
    assert np.max(np.abs(_flat(rho) - _flat(oracle.boltzmann(f.F)))) <= 1e-9 * v.max()


def test_equilibration_limits(oracle):
    """The step cap is honoured, and a Boltzmann start is already converged at the first
    check (its one-step change is rounding only)."""
    f = synth.random_fields((6, 5, 4), seed=43)
    rho, steps, res = oracle.equilibrate(f.F, 7, 0.0)
    assert steps == 7 and res > 0
    eq = oracle.boltzmann(f.F)
    rho, steps, res = oracle.equilibrate(f.F, 1000, 1e-14, rho=eq)
    assert steps == 1 and res <= 1e-14


# --------------------------------------------------------------------- P8 no hopping

def test_no_hop_limit(oracle):
    """p0 = 0: each site only precesses, G(n) = sum_i m_i(0) exp(i n theta_i)."""
    f = synth.random_fields((4, 3, 5), seed=31, delta_scale=7.0)
    n = 500
    res = oracle.run(f.F, f.delta, f.region, 1, n, p0=0.0)
    theta = brute.phases(f.delta, DT, NU0)
    want = np.exp(1j * np.outer(np.arange(n + 1), theta)).sum(axis=1)
    assert np.max(np.abs(res.fid() - want)) <= 1e-13 * f.n_sites


# --------------------------------------------------------------------- P9 continuous limit

def test_continuous_time_limit(oracle):
    """p0 -> eps p0 and theta -> eps theta: the chain tends to expm(t (Q + i Theta)), error O(eps)."""
    f = synth.random_fields((4, 4, 4), seed=37, F_scale=1.0, delta_scale=6.0)
    t = 50.0
    theta = brute.phases(f.delta, DT, NU0)
    T_ref, _, _ = brute.matrices((4, 4, 4), (PER, PER, PER), f.F, P0)
    exact = brute.expm_fid(T_ref, theta, np.ones(64), t)
    errs = []
    for eps in (0.1, 0.05, 0.025):
        n = int(round(t / eps))
        res = oracle.run(f.F, f.delta * eps, f.region, 1, n, p0=P0 * eps, moments=False)
        errs.append(abs(res.fid()[-1] - exact) / abs(exact))
    assert errs[0] < 5e-2
    for a, b in zip(errs, errs[1:]):
        assert 1.7 < a / b < 2.3     # first order in eps


# --------------------------------------------------------------------- P10 symmetry

def test_symmetry_invariance(oracle):
    """Reflections, axis permutations and periodic translations of the inputs leave G, the mass
    and the uptake unchanged and permute the MSD axes (periodic boundaries)."""
    f = synth.random_fields((6, 5, 4), seed=41, F_scale=1.0, n_regions=2)
    n = 150
    base = oracle.run(f.F, f.delta, f.region, 2, n)

    def check(F, d, r, perm):
        res = oracle.run(F, d, r, 2, n)
        assert rel_l2(res.fid(), base.fid()) <= 1e-12
        np.testing.assert_allclose(res.uptake(), base.uptake(), rtol=1e-12)
        np.testing.assert_allclose(res.msd(), base.msd()[:, perm], rtol=1e-12)

    # reflection in x (array axis 2)
    check(f.F[:, :, ::-1].copy(), f.delta[:, :, ::-1].copy(), f.region[:, :, ::-1].copy(), [0, 1, 2])
    # periodic translation
    sh = (1, 2, 3)
    check(np.roll(f.F, sh, (0, 1, 2)), np.roll(f.delta, sh, (0, 1, 2)),
          np.roll(f.region, sh, (0, 1, 2)), [0, 1, 2])
    # swap x and z: new array axes (x, y, z) <- old (z, y, x); new x is old z
    tr = (2, 1, 0)
    check(np.ascontiguousarray(f.F.transpose(tr)), np.ascontiguousarray(f.delta.transpose(tr)),
          np.ascontiguousarray(f.region.transpose(tr)), [2, 1, 0])


# --------------------------------------------------------------------- P11 linearity

def test_linearity_in_magnetisation(oracle):
    """G is linear in m(0) for fixed populations (Eq. (13) is a linear recursion)."""
    f = synth.random_fields((5, 4, 3), seed=43, F_scale=1.0, delta_scale=6.0)
    n = 120
    rng = np.random.default_rng(7)
    N = f.n_sites
    rho = np.ones(N)
    z = np.zeros(3 * N)
    a = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    c1, c2 = 0.7, -1.9

    def G(m):
        return oracle.run(f.F, f.delta, f.region, 1, n,
                          state=(rho, m.real.copy(), m.imag.copy(), z, z)).fid()

    assert rel_l2(G(c1 * a + c2 * b), c1 * G(a) + c2 * G(b)) <= 1e-12


# --------------------------------------------------------------------- P12 closed faces

def test_closed_axis_free_lattice(oracle):
    """Closed x: the two wall planes lose their outward attempt, MSD_x(1) = 2 p0 (1 - 1/nx);
    later MSD_x stays below 2 p0 n while y and z keep the free value; mass is exact."""
    for nx in (4, 9):
        F = np.zeros((3, 5, nx))
        res = oracle.run(F, np.zeros_like(F), np.zeros(F.shape, np.uint8), 1, 60,
                         bc=(CLO, PER, PER))
        msd = res.msd()
        assert abs(msd[1, 0] - 2 * P0 * (1 - 1 / nx)) <= 1e-14
        n = np.arange(61)
        assert np.all(msd[1:, 0] < 2 * P0 * n[1:])
        np.testing.assert_allclose(msd[:, 1], 2 * P0 * n, rtol=1e-12)
        np.testing.assert_allclose(msd[:, 2], 2 * P0 * n, rtol=1e-12)
        assert np.max(np.abs(res.mass() / res.mass()[0] - 1)) <= 1e-13


# --------------------------------------------------------------------- restart

def test_restart_is_bitwise(oracle):
    """N + M steps in one run equal N steps, then M steps from the saved state."""
    f = synth.random_fields((5, 6, 4), seed=47, F_scale=1.0, n_regions=2)
    full = oracle.run(f.F, f.delta, f.region, 2, 70)
    a = oracle.run(f.F, f.delta, f.region, 2, 30)
    b = oracle.run(f.F, f.delta, f.region, 2, 40, state=(a.rho, a.re, a.im, a.M1, a.M2))
    assert np.array_equal(full.records[30:], b.records)
    assert np.array_equal(full.rho, b.rho) and np.array_equal(full.im, b.im)
    assert np.array_equal(full.M2, b.M2)


# --------------------------------------------------------------------- P10 obstacles, link
# mobility, reservoir faces (section 2.1 and Fig. 1; after Eq. (7); section 3.2)

INF = math.inf
RES = 2


def _obstacles(shape_zyx, frac, seed):
    rng = np.random.default_rng(seed)
    return rng.random(shape_zyx) < frac


def test_enclosed_site_only_precesses(oracle):
    """A single accessible site walled in by obstacles: every attempt is rejected (Fig. 1),
    so its population stays and its magnetisation only precesses, G(n) = exp(i n theta)."""
    f = synth.random_fields((3, 3, 3), seed=71, delta_scale=5.0)
    F = np.full((3, 3, 3), INF)
    F[1, 1, 1] = 0.3
    n = 300
    res = oracle.run(F, f.delta, f.region, 1, n)
    theta = brute.phases(f.delta, DT, NU0)[13]
    assert np.allclose(res.mass(), 1.0, rtol=0, atol=1e-15)
    assert np.max(np.abs(res.fid() - np.exp(1j * theta * np.arange(n + 1)))) <= 1e-12
    assert np.all(res.s2() == 0.0)


def test_channel_is_one_dimensional(oracle):
    """A straight periodic channel of accessible sites through the solid: free 1-D diffusion
    along it (MSD_x = 2 p0 n, Eq. (7) with d = 1) and no spread across it."""
    F = np.full((5, 5, 16), INF)
    F[2, 2, :] = 0.0
    z = np.zeros_like(F)
    n = 400
    res = oracle.run(F, z, z.astype(np.uint8), 1, n)
    msd = res.msd()
    assert np.allclose(msd[:, 0], 2 * P0 * np.arange(n + 1), rtol=1e-12, atol=1e-12)
    assert np.all(msd[:, 1:] == 0.0)
    assert np.allclose(res.mass(), 16.0, rtol=1e-14)


def test_one_step_msd_with_obstacles_eq5(oracle):
    """Eq. (5) with p_acc = 0 towards obstacles: from a uniform start on a flat landscape
    the one-step <dx^2> is p0 times the accessible x-links per accessible site, counted
    directly on the mask."""
    mask = _obstacles((6, 7, 8), 0.3, 73)
    F = np.where(mask, INF, 0.0)
    z = np.zeros(F.shape)
    res = oracle.run(F, z, z.astype(np.uint8), 1, 1, bc=(PER, CLO, PER))
    open_ = ~mask
    for a, ax in ((0, 2), (1, 1), (2, 0)):
        links = 0
        for sh in (+1, -1):
            nb = np.roll(open_, -sh, axis=ax)
            ok = open_ & nb
            if a == 1:                     # closed y: no link across the faces
                edge = np.zeros_like(ok)
                if sh > 0:
                    edge[:, -1, :] = True
                else:
                    edge[:, 0, :] = True
                ok &= ~edge
            links += ok.sum()
        assert abs(res.msd()[1, a] - P0 * links / open_.sum()) <= 1e-15


@pytest.mark.parametrize("bc", [(PER, PER, PER), (CLO, PER, CLO)])
def test_obstacles_mobility_dense_brute_force(oracle, bc):
    """Random obstacles, random free energies and random per-site mobility on 4^3: FID and
    moments equal the dense matrices built link by link with alpha_ij = min(mu_i, mu_j)."""
    f = synth.random_fields((4, 4, 4), seed=75, F_scale=1.2, delta_scale=6.0)
    mask = _obstacles((4, 4, 4), 0.25, 75)
    F = np.where(mask, INF, f.F)
    mu = np.random.default_rng(76).uniform(0.2, 1.0, size=(4, 4, 4))
    n = 60
    res = oracle.run(F, f.delta, f.region, 1, n, bc=bc, mobility=mu)
    theta = brute.phases(f.delta, DT, NU0)
    m0 = (~mask).reshape(-1).astype(np.float64)
    T0, _, _ = brute.matrices((4, 4, 4), bc, F, P0, mobility=mu)
    assert rel_l2(res.fid(), brute.fid(T0, theta, m0, n)) <= 1e-12
    for a in range(3):
        T0a, T1a, T2a = brute.matrices((4, 4, 4), bc, F, P0, axis=a, mobility=mu)
        mom = brute.moments(T0a, T1a, T2a, m0, n)
        assert np.allclose(res.s1()[:, a], mom[:, 1], rtol=0, atol=1e-12)
        assert np.allclose(res.s2()[:, a], mom[:, 2], rtol=1e-12, atol=1e-12)
    assert np.all(res.rho[mask.reshape(-1)] == 0.0)


def test_boltzmann_stationary_with_obstacles_and_mobility(oracle):
    """Detailed balance survives a symmetric link factor (after Eq. (7)) and obstacles: one
    step from Eq. (2) (zero on obstacles, normalised to the accessible sites) changes
    nothing beyond rounding."""
    f = synth.random_fields((9, 7, 6), seed=77, F_scale=1.5)
    mask = _obstacles((6, 7, 9), 0.2, 77)
    F = np.where(mask, INF, f.F)
    mu = np.random.default_rng(78).uniform(0.05, 1.0, size=F.shape)
    eq = oracle.boltzmann(F)
    assert abs(eq.sum() - (~mask).sum()) <= 1e-12 * eq.sum()
    res = oracle.run(F, f.delta, f.region, 1, 3, bc=(CLO, PER, CLO), init="boltzmann",
                     mobility=mu)
    assert np.max(np.abs(res.rho - eq.reshape(-1))) <= 1e-14 * eq.max()


def test_uniform_mobility_scales_free_diffusion(oracle):
    """Eq. (7): a uniform factor c on every link scales alpha, hence the free-lattice MSD
    slope, to 2 p0 c per axis."""
    z = np.zeros((6, 5, 7))
    c = 0.37
    res = oracle.run(z, z, z.astype(np.uint8), 1, 50, mobility=np.full(z.shape, c))
    n = np.arange(51)
    for a in range(3):
        assert np.allclose(res.msd()[:, a], 2 * P0 * c * n, rtol=1e-12, atol=1e-13)


def test_reservoir_equilibrium_closed_form(oracle):
    """Reservoir faces at one chemical potential (rho_g = K exp(-F_g) on every face) fix
    the equilibrium to rho_i = K exp(-F_i) by detailed balance across the ghost links;
    the equilibration reaches it from an empty lattice."""
    f = synth.random_fields((5, 4, 6), seed=79, F_scale=0.8)
    K = 2.5
    res_faces = {}
    for axis in (0, 2):
        for side in (0, 1):
            Fg = 0.3 * (axis - 1) + 0.2 * side
            res_faces[(axis, side)] = (Fg, K * math.exp(-Fg), 0.0, 0.0)
    rho, steps, r = oracle.equilibrate(f.F, 200000, 1e-13, bc=(RES, PER, RES),
                                       rho=np.zeros(f.F.shape), reservoir=res_faces)
    assert r <= 1e-13
    want = K * np.exp(-f.F)
    assert np.max(np.abs(rho - want)) <= 1e-10 * want.max()


def test_reservoir_chain_linear_profile(oracle):
    """A flat 1-D chain of n sites between two reservoirs (rho_L, rho_R) carries a steady
    current, and its steady state is the linear profile through the ghosts:
    rho(z) = rho_L + (rho_R - rho_L) (z + 1) / (n + 1)."""
    n = 9
    F = np.zeros((n, 1, 1))
    rl, rr = 3.0, 0.5
    rho, steps, r = oracle.equilibrate(F, 400000, 1e-14, bc=(CLO, CLO, RES),
                                       reservoir={(2, 0): (0.0, rl, 0.0, 0.0),
                                                  (2, 1): (0.0, rr, 0.0, 0.0)})
    want = rl + (rr - rl) * (np.arange(n) + 1) / (n + 1)
    assert np.max(np.abs(rho.reshape(-1) - want)) <= 1e-11


@pytest.mark.parametrize("bc", [(RES, PER, CLO), (PER, RES, RES)])
def test_reservoir_dense_affine(oracle, bc):
    """Reservoir faces with magnetised ghosts, obstacles and mobility: population, FID and
    moments equal the dense affine system (ghost links as a source term)."""
    f = synth.random_fields((4, 3, 3), seed=81, F_scale=1.0, delta_scale=4.0)
    mask = _obstacles((3, 3, 4), 0.2, 81)
    F = np.where(mask, INF, f.F)
    mu = np.random.default_rng(82).uniform(0.3, 1.0, size=F.shape)
    rng = np.random.default_rng(83)
    faces = {}
    for axis in range(3):
        if bc[axis] == RES:
            for side in (0, 1):
                faces[(axis, side)] = (rng.normal(0, 1), rng.uniform(0.5, 2), rng.normal(),
                                       rng.normal())
    n = 40
    res = oracle.run(F, f.delta, f.region, 1, n, bc=bc, mobility=mu, reservoir=faces)
    gh = oracle.ghosts(faces)
    theta = brute.phases(f.delta, DT, NU0)
    rho0 = (~mask).reshape(-1).astype(np.float64)
    for a in range(3):
        T0, T1, T2, src = brute.matrices((4, 3, 3), bc, F, P0, axis=a, mobility=mu, ghost=gh)
        out = brute.run_affine(T0, T1, T2, src, theta, rho0, rho0, n)
        assert np.allclose(res.mass(), out[:, 0].real, rtol=1e-12, atol=0)
        assert rel_l2(res.fid(), out[:, 1]) <= 1e-12
        assert np.allclose(res.s1()[:, a], out[:, 2].real, rtol=0, atol=1e-11)
        assert np.allclose(res.s2()[:, a], out[:, 3].real, rtol=1e-12, atol=1e-11)
    assert abs(res.mass()[-1] - res.mass()[0]) > 1e-3          # the faces exchange matter
