"""Diagnostics, watchdog and run(t_end) of the C ABI on the GPU.

The wetted length on the y- wall and the height of the condensed phase on the
middle column (the spreading diameter D and the bounce height H_b of Sec. 3.5,
Tables 6-7), the extremes of C and the integrals are compared with the same
definitions evaluated in numpy on the FP64 oracle's state after the same steps.
"""
import math

import numpy as np
import pytest

from paper_2507_03366_amd import eulbfs as E
from paper_2507_03366_amd import problems as PB

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    E.lib()
    yield


def _reference(pr, W):
    """The diagnostics written out on a state W (5 planes) from the oracle."""
    wx, wy = PB.widths(pr)
    C = W[4]
    Cc = np.clip(C, 0.0, 1.0)
    return {"c_min": C.min(), "c_max": C.max(), "wetted_length": float((Cc[0, :] * wx).sum()),
            "axis_height": float((Cc[:, pr.nx // 2] * wy).sum())}


def _impact():
    return PB.impact_droplet(n=64, we=20.0, re=200.0)


def _spreading():
    """A half disc of radius 16 on a cold 55 deg wall: it spreads and freezes."""
    pr, st = PB.static_droplet(n=64, R=16, sigma=0.015625)
    walls = dict(pr.walls)
    w = walls["y-"]
    walls["y-"] = PB.Wall(w.flow, w.heat, w.T_w, 55.0)
    return pr.replace(walls=walls), st


def _graded_drop():
    wx = PB.graded_widths(60, 0.6, 1.04, 1.5, both_ends=True)
    wy = PB.graded_widths(45, 0.6, 1.05, 1.5)
    pr = PB.Problem(nx=60, ny=45, x_width=wx, y_width=wy, rho=(0.917, 1.0, 0.01), mu=(0.05, 0.05, 0.0005),
                    lam=(0.4, 0.4, 0.004), latent=10.0, sigma=0.005, gy=-1e-5, delta_t=0.3, dt=0.3,
                    walls={"y-": PB.Wall(PB.NOSLIP, PB.DIRICHLET, -1.0, 75.0), "y+": PB.Wall(PB.FREESLIP),
                           "x-": PB.Wall(), "x+": PB.Wall()})
    X, Y = PB.cell_centres(pr)
    st = PB.uniform_state(pr, T0=0.1)
    st.C = PB.droplet_profile(X, Y, 0.5 * wx.sum(), 0.0, 15.0, pr.xi)
    return pr, st


@pytest.mark.parametrize("case,steps", [("spreading", 600), ("graded", 300)])
def test_spreading_and_bounce_diagnostics_match_oracle(oracle, case, steps):
    """A drop spreading and freezing on a cold wall (uniform mesh) and a sessile
    drop on a graded mesh: the wetted length, the axis height and the extremes
    of C equal the oracle's state's to 1e-10, the integrals to 1e-10."""
    pr, st = _spreading() if case == "spreading" else _graded_drop()
    oracle.set_threads(16)
    Wref, _ = oracle.run(pr, st, steps)
    ref = _reference(pr, Wref)
    dref = oracle.diagnostics(pr, Wref)
    s = E.Solver(pr, st)
    try:
        s.run(steps)
        d = s.diagnostics()
    finally:
        s.close()
    for k in ("wetted_length", "axis_height"):
        assert d[k] == pytest.approx(ref[k], rel=1e-10), k
        assert d[k] > 1.0
    assert d["c_min"] == pytest.approx(ref["c_min"], abs=1e-12)
    assert d["c_max"] == pytest.approx(ref["c_max"], abs=1e-12)
    for k, i in (("mass", 0), ("volume_C", 1), ("enthalpy", 2), ("solid", 3)):
        assert d[k] == pytest.approx(dref[i], rel=1e-10), k


def test_diagnostics_of_a_sessile_half_disc():
    """The definitions themselves on the initial half disc of radius R = 16
    centred on the wall: the wetted length is the chord 2 sqrt(R^2 - 1/4) of the
    first row and the axis height is R, both within 0.05 cell (the tanh profile
    of Eq. 62 is odd about C = 1/2); the impact drop, 2 xi above the wall, wets
    nothing."""
    pr, st = PB.static_droplet(n=64, R=16, sigma=0.015625)
    s = E.Solver(pr, st)
    try:
        d = s.diagnostics()
    finally:
        s.close()
    assert d["wetted_length"] == pytest.approx(2.0 * math.sqrt(16.0 ** 2 - 0.25), abs=0.05)
    assert d["axis_height"] == pytest.approx(16.0, abs=0.05)
    pr, st = _impact()
    s = E.Solver(pr, st)
    try:
        d = s.diagnostics()
    finally:
        s.close()
    assert d["wetted_length"] < 0.05
    assert d["axis_height"] == pytest.approx(pr.nx / 4.0, abs=0.1)  # the diameter D = n/4


def test_order_parameter_out_of_range_is_reported():
    """The watchdog: a state whose C leaves [-0.5, 1.5] is reported by a
    diagnostics query (output still written) and by run; a checkpoint restores
    the handle."""
    pr, st = PB.static_droplet(n=64, R=16, sigma=0.015625)
    s = E.Solver(pr, st)
    try:
        good = s.conserved()
        bad = good.copy()
        bad[4, 10, 20] = 1.8
        s.set_conserved(bad)
        with pytest.raises(E.EulbfsError) as ei:
            s.diagnostics()
        assert ei.value.code == E.EUNSTABLE and "order parameter" in str(ei.value)
        out = np.zeros(E.NDIAG)
        rc = E.lib().eulbfs_query(s.h, E.SCALAR_DIAG, out.ctypes.data_as(__import__("ctypes").c_void_p),
                                  out.nbytes, 0)
        assert rc == E.EUNSTABLE and out[11] == pytest.approx(1.8)
        with pytest.raises(E.EulbfsError):
            s.conserved()  # a poisoned handle reports on every query
        s.set_conserved(good)
        s.run(5)
        assert s.diagnostics()["c_max"] < 1.5
    finally:
        s.close()


def test_run_stops_at_t_end():
    """run(nsteps, t_end) takes the steps that bring the time to t_end at most:
    ceil((t_end - t)/dt) of them; t_end already reached takes none; NaN is
    rejected."""
    pr, st = PB.conductive_freezing()
    s = E.Solver(pr, st)
    try:
        s.run(1000, t_end=5.0)  # dt = 0.5
        assert s.diagnostics()["steps"] == 10
        s.run(1000, t_end=5.0)
        assert s.diagnostics()["steps"] == 10
        s.run(1000, t_end=6.2)
        assert s.diagnostics()["steps"] == 13
        s.run(4)
        d = s.diagnostics()
        assert d["steps"] == 17 and d["time"] == pytest.approx(8.5)
        with pytest.raises(E.EulbfsError) as ei:
            s.run(3, t_end=float("nan"))
        assert ei.value.code == E.EINVAL
    finally:
        s.close()
