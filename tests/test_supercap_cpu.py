"""Host side of the supercapacitor workflow (section 4): the synthetic systems and the
per-part diffusion coefficients of the C ABI, on the CPU."""
import numpy as np
import pytest

from paper_2603_22553_amd import supercap as S

SMALL = dict(shape_xyz=(24, 20, 60), electrode=20, radius=4)


@pytest.mark.parametrize("kind", ["monolith", "film"])
def test_structure(kind):
    s = S.system(kind, 0.0, **SMALL)
    f, r = s.fields, s.fields.region
    assert f.F.shape == (60, 20, 24) and f.n_regions == 3
    assert np.all(r[:20] == S.NEGATIVE) and np.all(r[40:] == S.POSITIVE) and np.all(r[20:40] == S.BULK)
    assert not s.carbon[r == S.BULK].any()
    assert np.all(f.F[~s.carbon] == 0.0) and np.all(f.delta[~s.carbon] == 0.0)
    assert np.all(f.F[s.carbon] < 0.0) and np.all(f.delta[s.carbon] < 0.0)
    frac = s.carbon[r != S.BULK].mean()
    if kind == "monolith":
        assert frac == 1.0
    else:
        assert 0.38 <= s.carbon[r == S.NEGATIVE].mean() < 0.45
        assert 0.38 <= s.carbon[r == S.POSITIVE].mean() < 0.45
    assert f.periodic == (True, True, False)


def test_potential_moves_anions_and_shifts():
    """Per volt, on carbon sites only: F up by bias in the negative electrode, down in the
    positive one, shifts up by shift_ppm; the carbon structure is the same at both
    potentials."""
    a = S.system("film", 0.0, bias=0.3, shift_ppm=1.5, **SMALL)
    b = S.system("film", 2.0, bias=0.3, shift_ppm=1.5, **SMALL)
    r = a.fields.region
    assert np.array_equal(a.carbon, b.carbon)
    dF = b.fields.F - a.fields.F
    c = a.carbon
    assert np.allclose(dF[c & (r == S.NEGATIVE)], 0.6) and np.allclose(dF[c & (r == S.POSITIVE)], -0.6)
    assert np.all(dF[~c] == 0.0)          # bulk and the bulk-like sites between particles
    dd = b.fields.delta - a.fields.delta
    assert np.allclose(dd[a.carbon], 3.0) and np.all(dd[~a.carbon] == 0.0)


def test_region_diffusion_closed_form():
    """lpc_region_diffusion (host-only, through the C ABI) on free-lattice moments: the MSD
    grows by 2 p0 per step and axis (Eq. (7)), so D / D_bulk = 1 and D = p0 a^2 / dt."""
    from paper_2603_22553_amd.lattice import region_diffusion
    p0, dt, a = 1.0 / 240.0, 5e-6, 0.5e-9
    rho = np.array([5.0, 7.0, 11.0])

    def table(t):
        m = np.zeros((3, 7))
        m[:, 0] = rho
        m[:, 4:7] = rho[:, None] * 2 * p0 * t
        return m

    D, ratio = region_diffusion(table(100), table(350), 250, p0, dt, a, axes=(0, 1))
    assert np.allclose(ratio, 1.0, rtol=1e-14)
    assert np.allclose(D, p0 * a * a / dt, rtol=1e-14)
    # part 1 diffuses at half speed in the plane; z is not averaged in
    slow = table(350)
    slow[1, 4:6] = rho[1] * (2 * p0 * 100 + 0.5 * 2 * p0 * 250)
    slow[1, 6] = 0.0
    _, ratio = region_diffusion(table(100), slow, 250, p0, dt, a, axes=(0, 1))
    assert np.isclose(ratio[1], 0.5, rtol=1e-14) and np.allclose(ratio[[0, 2]], 1.0)
    # one axis alone, and a population that changed between the tables (the MSD is per
    # particle now in the part)
    moved = table(350)
    moved[2] *= 2.0
    _, ratio = region_diffusion(table(100), moved, 250, p0, dt, a, axes=(2,))
    assert np.allclose(ratio, 1.0, rtol=1e-14)


def test_region_diffusion_errors():
    from paper_2603_22553_amd import _native as N
    from paper_2603_22553_amd.lattice import region_diffusion
    t = np.ones((2, 7))
    empty = t.copy()
    empty[1, 0] = 0.0
    for kw, status in ((dict(axes=()), N.LPC_ERR_ARG), (dict(steps_between=0), N.LPC_ERR_ARG),
                       (dict(p_hop=0.0), N.LPC_ERR_ARG), (dict(sums_b=empty), N.LPC_ERR_STATE)):
        args = dict(sums_a=t, sums_b=t, steps_between=10, p_hop=1 / 7)
        args.update(kw)
        with pytest.raises(N.LpcError) as e:
            region_diffusion(**args)
        assert e.value.status == status
