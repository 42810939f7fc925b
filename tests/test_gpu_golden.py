"""The hand-derived golden cases (tests/golden/hand_cases.json) on the GPU path, through the
C ABI: exact fractions worked out from Eqs. (1) and (13), moment propagation, inaccessible
sites, link mobility and Dirichlet ghost sites, compared without the oracle in between."""
import numpy as np
import pytest

from conftest import load_golden, parse_value

pytestmark = pytest.mark.gpu

# The mixed path stores the phase per step in float: a phase near 2 pi is quantised to half an
# ulp of about 6, 2.4e-7, which moves m by as much; 1e-6 leaves four such ulps.
TOL = {"fp64": 1e-14, "mixed": 1e-6}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", load_golden("hand_cases.json")["cases"], ids=lambda c: c["name"])
def test_hand_case_on_gpu(case, precision):
    from paper_2603_22553_amd.lattice import Lattice
    nx, ny, nz = case["shape_xyz"]
    shape = (nz, ny, nx)
    vals = lambda key: np.array([parse_value(v) for v in case[key]]).reshape(shape)
    tol = TOL[precision]
    for step in case["steps"]:
        with Lattice(case["shape_xyz"], bc=tuple(case["bc"]), precision=precision,
                     n_regions=case["n_regions"], p_hop=parse_value(case["p0"]),
                     dt_s=case["dt"], larmor_hz=case["nu0"], max_records=step["n"] + 1,
                     mobility="mobility" in case) as lat:
            lat.set_free_energy(vals("F"))
            lat.set_shift(vals("delta_ppm"))
            lat.set_regions(np.array(case["region"], dtype=np.uint8).reshape(shape))
            if "mobility" in case:
                lat.set_mobility(vals("mobility"))
            for key, g in case.get("reservoir", {}).items():
                axis, side = (int(v) for v in key.split(","))
                F, rho, re, im = (parse_value(v) for v in g)
                lat.set_reservoir(axis, side, F, rho, complex(re, im))
            init = case.get("init", "uniform")
            if isinstance(init, str):
                lat.init_state(init)
            else:
                lat.init_state(rho=vals("init"))
            lat.run(step["n"])
            rho = lat.population().reshape(-1)
            m = lat.magnetization().reshape(-1)
            rec = lat.records()[-1]
        want = {k: np.array([parse_value(v) for v in step[k]]) for k in
                ("rho", "m_re", "m_im", "S1", "S2")}
        R = case["n_regions"]
        assert np.allclose(rho, want["rho"], rtol=0, atol=tol), (case["name"], step["n"], "rho")
        assert np.allclose(m.real, want["m_re"], rtol=0, atol=tol), (case["name"], "m_re")
        assert np.allclose(m.imag, want["m_im"], rtol=0, atol=tol), (case["name"], "m_im")
        assert np.allclose(rec[3 * R:3 * R + 3], want["S1"], rtol=0, atol=tol), (case["name"], "S1")
        assert np.allclose(rec[3 * R + 3:3 * R + 6], want["S2"], rtol=0, atol=tol), (case["name"], "S2")
