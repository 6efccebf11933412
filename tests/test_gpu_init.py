"""Closed-form initial states built on the device (EULBFS_INIT_ANALYTIC)
against the same states built on the host by problems.Shape: every stored
field within a few units in the last place (the device and the host each
evaluate tanh with their own library), on uniform and stretched meshes, in
FP64 and FP32 mode, for a solver and for a batch request."""
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


def _graded_layer():
    pr, st = PB.three_phase_stefan(nx=80, ny=6)
    wx = PB.graded_widths(80, 0.6, 1.03, 1.4)
    pr = pr.replace(x_width=wx, delta_t=0.3, dt=0.3)
    return pr, PB.Shape(profile=PB.PROFILE_LAYER, axis=0, h0=30.0, t_out=0.05, t_in=-0.02).state(pr)


def _graded_drop():
    pr, _ = PB.static_droplet(n=64, R=16, sigma=0.015625)
    wx = PB.graded_widths(64, 0.6, 1.04, 1.5, both_ends=True)
    wy = PB.graded_widths(64, 0.6, 1.05, 1.5)
    pr = pr.replace(x_width=wx, y_width=wy, delta_t=0.3, dt=0.3)
    sh = PB.Shape(profile=PB.PROFILE_DROPLET, x0=0.5 * wx.sum(), y0=0.0, r0=15.0, t_amp=1e-3, seed=11, v_in=-0.01)
    return pr, sh.state(pr)


CASES = {
    "conductive": lambda: PB.conductive_freezing(),
    "stefan3": lambda: PB.three_phase_stefan(),
    "full_freezing": lambda: PB.stefan_full_freezing(0.8, ny=4),
    "film_noise": lambda: PB.film_freezing(n=96),
    "droplet": lambda: PB.static_droplet(n=128, R=32, sigma=0.015625),
    "impact": lambda: PB.impact_droplet(n=96),
    "film_table1": lambda: PB.film_table1(1.0, nx=50, ny=100, H0=25.0),
    "table3": lambda: PB.table3_droplet("water", 120.0, nx=100, ny=50, R=12.5,
                                        sigma=PB.table3_droplet("water", 120.0)[0].sigma),
    "graded_layer": _graded_layer,
    "graded_drop": _graded_drop,
}


def _close(a, b):
    scale = max(1.0, float(np.abs(b).max()))
    return float(np.abs(a - b).max()) <= 8e-16 * scale


@pytest.mark.parametrize("precision", [E.FP64, E.FP32])
@pytest.mark.parametrize("case", list(CASES))
def test_device_built_state_equals_host_built(case, precision):
    pr, st = CASES[case]()
    assert st.shape is not None
    host = E.Solver(pr, st, precision=precision)
    dev = E.Solver(pr, st, precision=precision, analytic=True)
    try:
        for name in ("C", "T", "FL", "U", "V", "P", "H"):
            a, b = dev.field(name), host.field(name)
            if precision == E.FP32 and name in ("U", "V", "P"):
                assert np.abs(a - b).max() <= 2.0 ** -22 * float(np.abs(b).max()), name
            else:
                assert _close(a, b), (name, float(np.abs(a - b).max()))
        if case in ("film_noise", "graded_drop"):
            assert np.abs(dev.field("T")).max() > 0  # the seeded noise is there
    finally:
        host.close()
        dev.close()


def test_batch_admits_a_shape():
    """A batch request built on the device from its shape: the same state as
    the host-built request to rounding, and bitwise the same state as a solver
    built from the same shape after 50 steps."""
    import torch

    pr, st = PB.impact_droplet(n=64)
    b = E.Batch(1 << 27, 4, precision=E.FP64, stream=torch.cuda.Stream())
    try:
        s_dev = b.admit(pr, st, 50, analytic=True)
        s_host = b.admit(pr, st, 50)
        w_dev0, w_host0 = b.conserved(s_dev), b.conserved(s_host)
        for k in range(5):
            assert _close(w_dev0[k], w_host0[k]), k
        while b.diagnostics(s_dev)["steps"] < 50:
            b.tick(25)
        w_dev = b.conserved(s_dev)
    finally:
        b.close()
    s = E.Solver(pr, st, kernel=E.KERNEL_AUTO, analytic=True)
    try:
        s.run(50)
        assert np.array_equal(s.conserved(), w_dev)
    finally:
        s.close()


@pytest.mark.parametrize("case", ["impact", "film_noise"])
def test_device_built_state_runs_like_the_oracle(oracle, case):
    """Started from the device-built fields, 500 steps stay within 1e-10
    relative L2 per field of the oracle started from the host-built ones (the
    two starts differ in the last place of tanh at most)."""
    pr, st = CASES[case]()
    oracle.set_threads(16)
    Wref, _ = oracle.run(pr, st, 500)
    s = E.Solver(pr, st, kernel=E.KERNEL_AUTO, analytic=True)
    try:
        s.run(500)
        w = s.conserved()
    finally:
        s.close()
    for name, ks in (("H", [0]), ("p", [1]), ("M", [2, 3]), ("C", [4])):
        err = np.linalg.norm((w[ks] - Wref[ks]).ravel()) / np.linalg.norm(Wref[ks].ravel())
        assert err <= 1e-10, (name, err)
