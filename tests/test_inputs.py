"""The seeded input generators and closed-form initial states (CPU): the
splitmix64 generator against its published output sequence, and the
closed-form shapes against Eqs. (61) and (62) written out."""
import math

import numpy as np
import pytest

from paper_2507_03366_amd import problems as PB


def test_splitmix64_reference_sequence():
    """Seeded with 0, the generator's reference implementation returns
    0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f first: their
    top 53 bits scaled to [-1, 1)."""
    ref = (0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F)
    want = np.array([(r >> 11) * 2.0 ** -52 - 1.0 for r in ref])
    assert np.array_equal(PB.splitmix_uniform(0, np.array([1, 2, 3])), want)
    u = PB.splitmix_uniform(12345, np.arange(1, 200001))
    assert u.min() >= -1.0 and u.max() < 1.0 and abs(u.mean()) < 5e-3 and abs(u.var() - 1.0 / 3.0) < 5e-3


def test_shapes_follow_the_closed_forms():
    pr, st = PB.three_phase_stefan(nx=64, ny=2, H0=20.0)
    x = np.arange(64) + 0.5
    assert np.allclose(st.C[0], 0.5 * (1.0 + np.tanh(2.0 * (20.0 - x) / pr.xi)), rtol=0, atol=1e-15)
    assert st.shape.profile == PB.PROFILE_LAYER and st.shape.axis == 0
    pr, st = PB.impact_droplet(n=64)
    D = 16.0
    X, Y = PB.cell_centres(pr)
    r = np.hypot(X - 32.0, Y - (0.5 * D + 2.0 * pr.xi))
    assert np.allclose(st.C, 0.5 * (1.0 + np.tanh(2.0 * (0.5 * D - r) / pr.xi)), rtol=0, atol=1e-15)
    assert np.array_equal(st.T, np.where(st.C > 0.5, -0.5, 0.0))
    assert np.array_equal(st.v, -0.05 * st.C) and not st.u.any() and not st.p.any()
    pr, st = PB.film_freezing(n=32, seed=7, amp=1e-3)
    n = np.arange(1, 32 * 32 + 1).reshape(32, 32)
    assert np.array_equal(st.T, 1e-3 * PB.splitmix_uniform(7, n))
    # half disc of radius R: the C = 1/2 contour passes through (x0 +- R, 0)
    pr, st = PB.static_droplet(n=64, R=16.0, sigma=0.015625)
    assert st.shape.r0 == pytest.approx(16.0) and st.shape.y0 == pytest.approx(0.0, abs=1e-12)
    assert math.isclose(st.C[0, 32 + 15], 0.5 * (1.0 + math.tanh(2.0 * (16.0 - math.hypot(15.5, 0.5)) / pr.xi)),
                        abs_tol=1e-15)


def test_impact_case_b_follows_the_text():
    """The Sec. 3.5 case (b) parameters as printed (fixture
    tests/golden/impact_sec35.txt), and their dimensionless groups in the
    lattice problem: Re = 678, We = 6.67 and Pr = 12.8 from the Table 1 water."""
    import os

    g = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "impact_sec35.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split("=")
                g[k.strip()] = [float(x) for x in v.split()]
    c = PB.IMPACT_CASES["b"]
    assert [c["D"] * 1e3, c["U"], c["T_0"], c["T_w"], c["theta_adv"], c["theta_rec"], c["theta_eq"]] == \
        pytest.approx(g["case_b"])
    pr, st = PB.impact_sec35("b")
    U, D0 = 0.05, 100.0
    assert U * D0 / pr.mu[1] == pytest.approx(1000 * 0.44 * 2.62e-3 / 0.0017)
    assert U * U * D0 / pr.sigma == pytest.approx(1000 * 0.44 ** 2 * 2.62e-3 / 0.076)
    assert pr.mu[1] / pr.lam[1] == pytest.approx(0.0017 * 4210 / 0.56)
    assert 1.0 / pr.latent == pytest.approx(4210 * 30 / 334000)
    assert st.T.max() == pytest.approx(25.0 / 30.0) and st.v.min() == pytest.approx(-U)
    assert PB.impact_time("b", 0.015) == pytest.approx(0.015 * 0.44 / 2.62e-3 * D0 / U)
