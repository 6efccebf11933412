"""GPU (gfx950) vs FP64 CPU oracle: element-by-element parity through the C ABI.

Tolerances (FP64): face fluxes and residuals of one evaluation agree to
1e-12 of each component's largest magnitude (the two sides evaluate the same
formulas in a different order, with FMA contraction on the GPU); whole runs
agree to 1e-10 relative L2 per conserved field after 1000 steps (every
data-dependent branch of the method is continuous or static, so rounding
differences do not grow into O(1) differences).
"""
import math

import numpy as np
import pytest

from paper_2507_03366_amd import eulbfs as E
from paper_2507_03366_amd import problems as PB

pytestmark = pytest.mark.gpu

FIELDS = ("H", "p", "Mx", "My", "C")
# physical fields of W: the momentum (rho c_s^2 u, rho c_s^2 v) is one vector field
GROUPS = (("H", [0]), ("p", [1]), ("M", [2, 3]), ("C", [4]))


def rel_l2(a, b):
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / den) if den > 0 else float(np.linalg.norm(a.ravel()))


def field_errors(w, ref):
    """relative L2 per physical field; fields that are zero in the reference
    report the absolute norm of the GPU field instead"""
    return {name: rel_l2(w[ks], ref[ks]) for name, ks in GROUPS}


def scaled_err(a, b):
    """max |a - b| / max |b| per component (components along axis 0)."""
    out = []
    for k in range(a.shape[0]):
        s = np.abs(b[k]).max()
        out.append(np.abs(a[k] - b[k]).max() / s if s > 0 else np.abs(a[k]).max())
    return np.array(out)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    E.lib()
    yield


def _walls(flow, heat, theta, Tw=-1.0):
    return PB.Wall(flow, heat, Tw, theta)


def _cases():
    """Small grids covering every boundary rule, both h/g lattices, both
    surface-tension forms, gravity, ragged sizes and mushy closures."""
    cases = []
    base = dict(rho=(0.917, 1.0, 0.05), mu=(0.05, 0.04, 0.004), lam=(0.5, 0.4, 0.02), cp=(1.2, 1.0, 0.9),
                latent=3.0, sigma=0.02, mobility=0.08, gy=-1e-4)
    cases.append(("periodic9", PB.Problem(nx=8, ny=8, periodic_x=True, periodic_y=True, **base)))
    cases.append(("periodic5", PB.Problem(nx=8, ny=8, lattice_hg=5, periodic_x=True, periodic_y=True, **base)))
    cases.append(("walls_mixed", PB.Problem(nx=8, ny=8, walls={
        "x-": _walls(PB.NOSLIP, PB.DIRICHLET, 60.0), "x+": _walls(PB.FREESLIP, PB.ADIABATIC, 90.0),
        "y-": _walls(PB.NOSLIP, PB.DIRICHLET, 120.0, -0.5), "y+": _walls(PB.OUTLET, PB.ADIABATIC, 75.0)}, **base)))
    cases.append(("ragged_surf1", PB.Problem(nx=37, ny=13, surf_model=1, periodic_x=True, walls={
        "y-": _walls(PB.NOSLIP, PB.DIRICHLET, 70.0), "y+": _walls(PB.FREESLIP, PB.ADIABATIC, 100.0)}, **base)))
    cases.append(("mushy_dt", PB.Problem(nx=12, ny=9, T_s=-0.2, T_l=0.1, delta_t=0.3, periodic_y=True, walls={
        "x-": _walls(PB.NOSLIP, PB.DIRICHLET, 90.0), "x+": _walls(PB.NOSLIP, PB.ADIABATIC, 90.0)}, **base)))
    # one heat capacity for all phases (the uniform-C_p fast path), with and
    # without delta_t = dx/2, with a mushy range
    ucp = dict(base, cp=(1.1, 1.1, 1.1))
    cases.append(("ucp_dt_mushy", PB.Problem(nx=12, ny=9, T_s=-0.2, T_l=0.1, delta_t=0.3, periodic_y=True, walls={
        "x-": _walls(PB.NOSLIP, PB.DIRICHLET, 80.0), "x+": _walls(PB.NOSLIP, PB.ADIABATIC, 90.0)}, **ucp)))
    cases.append(("ucp_half_mushy", PB.Problem(nx=10, ny=11, T_s=-0.2, T_l=0.1, periodic_x=True, walls={
        "y-": _walls(PB.NOSLIP, PB.DIRICHLET, 110.0), "y+": _walls(PB.FREESLIP, PB.ADIABATIC, 90.0)}, **ucp)))
    # contact-angle hysteresis windows on every wall (seeded C straddles the
    # interface at the walls, so the apparent angles hit both bounds and the
    # inside of the windows)
    hw = {"x-": PB.Wall(PB.NOSLIP, PB.DIRICHLET, -1.0, 80.0, 100.0, 40.0),
          "x+": PB.Wall(PB.FREESLIP, PB.ADIABATIC, 0.0, 90.0, 95.0, 85.0),
          "y-": PB.Wall(PB.NOSLIP, PB.DIRICHLET, -0.5, 120.0, 150.0, 60.0),
          "y+": PB.Wall(PB.OUTLET, PB.ADIABATIC, 0.0, 70.0, 70.0, 70.0)}
    cases.append(("hysteresis", PB.Problem(nx=9, ny=10, walls=hw, **base)))
    return cases


CASES = _cases()


@pytest.mark.parametrize("name,pr", CASES, ids=[c[0] for c in CASES])
def test_ghost_ring_matches_oracle(oracle, name, pr):
    st = PB.seeded_fields(pr, seed=11)
    W = oracle.init(pr, st)
    s = E.Solver(pr, st)
    try:
        w6 = s.conserved()
        assert scaled_err(w6[:5], W).max() < 1e-14
        g = s.ghosted()
        ref = oracle.ghosts(pr, W)
        assert scaled_err(g, ref).max() < 1e-13, name
    finally:
        s.close()


@pytest.mark.parametrize("name,pr", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("kernel", [E.KERNEL_FUSED, E.KERNEL_SPLIT])
def test_fluxes_and_residual_match_oracle(oracle, name, pr, kernel):
    st = PB.seeded_fields(pr, seed=5)
    W = oracle.init(pr, st)
    fs = 0.01 * np.random.default_rng(3).uniform(-1, 1, (pr.ny, pr.nx))
    R_ref, Fx_ref, Fy_ref = oracle.residual(pr, W, fs)
    s = E.Solver(pr, st, kernel=kernel)
    try:
        w6 = s.conserved()
        w6[5] = fs
        s.set_conserved(w6)
        R, Fx, Fy = s.residual()
        assert scaled_err(Fx, Fx_ref).max() < 1e-12, (name, scaled_err(Fx, Fx_ref))
        assert scaled_err(Fy, Fy_ref).max() < 1e-12, (name, scaled_err(Fy, Fy_ref))
        assert scaled_err(R, R_ref).max() < 1e-11, (name, scaled_err(R, R_ref))
    finally:
        s.close()


@pytest.mark.parametrize("name,pr", CASES, ids=[c[0] for c in CASES])
def test_one_step_fused_and_split_match_oracle(oracle, name, pr):
    st = PB.seeded_fields(pr, seed=21, amp=0.5)
    Wref, fsref = oracle.run(pr, st, 3)
    out = []
    for kernel in (E.KERNEL_FUSED, E.KERNEL_SPLIT):
        s = E.Solver(pr, st, kernel=kernel)
        try:
            s.step(3)
            w6 = s.conserved()
        finally:
            s.close()
        errs = field_errors(w6[:5], Wref)
        assert max(errs.values()) < 1e-12, (name, kernel, errs)
        assert np.abs(w6[5] - fsref).max() <= 1e-12 * max(1.0, np.abs(fsref).max())
        out.append(w6)
    assert np.abs(out[0] - out[1]).max() <= 1e-13 * np.abs(out[1]).max()


def _parity_run(oracle, pr, st, steps, tol=1e-10, kernel=E.KERNEL_FUSED, tile=(0, 0)):
    oracle.set_threads(16)
    Wref, fsref = oracle.run(pr, st, steps)
    s = E.Solver(pr, st, kernel=kernel, tile=tile)
    try:
        s.step(steps)
        w6 = s.conserved()
        d = s.diagnostics()
    finally:
        s.close()
    errs = field_errors(w6[:5], Wref)
    assert max(errs.values()) <= tol, errs
    dref = oracle.diagnostics(pr, Wref)
    # the integrals are sums over up to 2.6e5 cells in a different order on
    # each side (two-pass wave reduction vs a sequential loop): n * eps ~ 3e-11
    assert d["mass"] == pytest.approx(dref[0], rel=1e-10)
    assert d["volume_C"] == pytest.approx(dref[1], rel=1e-10)
    assert d["enthalpy"] == pytest.approx(dref[2], rel=1e-10, abs=1e-12)
    assert d["solid"] == pytest.approx(dref[3], rel=1e-10, abs=1e-12)
    return w6, Wref, d


def test_conductive_freezing_full_size_1000_steps(oracle):
    """Sec. 3.1 configuration at its full size (128 x 4)."""
    pr, st = PB.conductive_freezing()
    w6, _, d = _parity_run(oracle, pr, st, 1000)
    assert np.all(w6[2] == 0) and np.all(w6[3] == 0) and np.all(w6[1] == 0)


def test_three_phase_stefan_full_size_1000_steps(oracle):
    """Sec. 3.2 configuration at its full size (256 x 8), rho_s/rho_l = 0.9."""
    pr, st = PB.three_phase_stefan()
    _parity_run(oracle, pr, st, 1000)


def test_film_reduced_1000_steps(oracle):
    """Sec. 3.3 configuration (cold bottom, gravity, noise) on a 64 x 64 grid."""
    pr, st = PB.film_freezing(n=64)
    _parity_run(oracle, pr, st, 1000)


def test_droplet_reduced_1000_steps_d2q5(oracle):
    """Sec. 3.4 configuration on 64 x 64 with the D2Q5 h/g lattice."""
    pr, st = PB.static_droplet(n=64, R=16, lattice_hg=5)
    pr = pr.replace(sigma=0.015625)
    _parity_run(oracle, pr, st, 1000)


def test_impact_reduced_1000_steps(oracle):
    """Sec. 3.5 configuration (moving supercooled drop, F_surf = -F_l C grad mu_c) on 64 x 64."""
    pr, st = PB.impact_droplet(n=64, we=20.0, re=200.0)
    _parity_run(oracle, pr, st, 1000)


@pytest.mark.parametrize("tile", [(32, 8), (64, 4), (16, 16), (64, 8), (32, 16), (32, 32)])
def test_tiles_agree_on_ragged_grid(oracle, tile):
    pr, st = PB.static_droplet(n=64, R=16)
    pr = pr.replace(nx=70, ny=45, sigma=0.015625)
    X, Y = PB.cell_centres(pr)
    st = PB.uniform_state(pr)
    st.C = PB.droplet_profile(X, Y, 35.0, 0.0, 16.0, 4.0)
    _parity_run(oracle, pr, st, 200, tol=1e-11, tile=tile)


def test_droplet_full_size_512(oracle):
    """Sec. 3.4 configuration at its full size (512 x 512, R = 128) in the launch
    configuration of the benchmark (fused kernel, tile picked by the autotuner):
    1000 steps, 1e-10 relative L2 per field and the integrals."""
    pr, st = PB.static_droplet()
    _parity_run(oracle, pr, st, 1000, kernel=E.KERNEL_AUTO)


def test_large_grid_2048(oracle):
    """2048 x 2048 (16384 tiles of 32 x 8, 4096 of 32 x 16: every XCD holds many
    tiles) in the autotuned configuration, two steps against the oracle."""
    pr, _ = PB.static_droplet(n=2048, R=512)
    X, Y = PB.cell_centres(pr)
    st = PB.uniform_state(pr)
    st.C = PB.droplet_profile(X, Y, 1024.0, 0.0, 512.0, 4.0)
    _parity_run(oracle, pr, st, 2, tol=1e-12, kernel=E.KERNEL_AUTO)


def test_periodic_tiling_at_8192(oracle):
    """A 64 x 64 periodic state tiled 128 x 128 times (8192 x 8192 = 67 M cells,
    65 536 tiles of 32 x 32): after three autotuned steps every 64 x 64 block on
    the GPU is the same bits as every other and matches the oracle's 64 x 64
    run to 1e-12 (an indexing or tile-mapping error anywhere in the large grid
    shows up as a block that differs)."""
    base = dict(rho=(0.917, 1.0, 0.05), mu=(0.05, 0.04, 0.004), lam=(0.5, 0.4, 0.02), cp=(1.2, 1.0, 0.9),
                latent=3.0, sigma=0.02, mobility=0.08, periodic_x=True, periodic_y=True)
    small = PB.Problem(nx=64, ny=64, **base)
    st = PB.seeded_fields(small, seed=5, amp=0.5)
    oracle.set_threads(16)
    Wref, _ = oracle.run(small, st, 3)
    reps = 128
    big = PB.Problem(nx=64 * reps, ny=64 * reps, **base)
    tiled = PB.InitialState(*(np.tile(a, (reps, reps)) for a in (st.T, st.Fl, st.C, st.u, st.v, st.p)))
    s = E.Solver(big, tiled, kernel=E.KERNEL_AUTO)
    del tiled
    try:
        s.step(3)
        w = s.conserved()[:5]
    finally:
        s.close()
    blocks = w.reshape(5, reps, 64, reps, 64)
    first = blocks[:, 0, :, 0, :]
    assert (blocks == first[:, None, :, None, :]).all()
    assert scaled_err(first, Wref).max() < 1e-12


def test_film_full_size_256(oracle):
    """Sec. 3.3 configuration at its full size (256 x 256, gravity, the seeded
    temperature noise): 1000 steps, 1e-10 relative L2 per field."""
    pr, st = PB.film_freezing()
    _parity_run(oracle, pr, st, 1000, kernel=E.KERNEL_AUTO)


def test_minimum_grid(oracle):
    pr = PB.Problem(nx=4, ny=4, rho=(0.9, 1.0, 0.1), mu=(0.05, 0.05, 0.005), lam=(0.4, 0.4, 0.04), latent=2.0,
                    sigma=0.01, walls={s: PB.Wall(PB.NOSLIP, PB.DIRICHLET if s == "y-" else PB.ADIABATIC, -1.0, 80.0)
                                       for s in PB.SIDES})
    st = PB.seeded_fields(pr, seed=2, amp=0.3)
    _parity_run(oracle, pr, st, 50, tol=1e-11)


def test_deterministic_and_checkpoint_restart():
    pr, st = PB.static_droplet(n=96, R=24)
    pr = pr.replace(sigma=0.015625)
    a = E.Solver(pr, st)
    a.step(40)
    w_a = a.conserved()
    a.close()
    b = E.Solver(pr, st)
    b.step(20)
    ck = b.conserved()
    b.close()
    c = E.Solver(pr, conserved=ck)
    c.step(20)
    w_c = c.conserved()
    c.close()
    d = E.Solver(pr, st)
    d.step(40)
    w_d = d.conserved()
    d.close()
    assert np.array_equal(w_a, w_d)
    assert np.array_equal(w_a, w_c)


def test_nonfinite_state_is_reported():
    pr, st = PB.conductive_freezing()
    s = E.Solver(pr, st)
    try:
        w6 = s.conserved()
        w6[0, 2, 5] = np.nan
        s.set_conserved(w6)
        with pytest.raises(E.EulbfsError) as ei:
            s.run(1)
        assert ei.value.code == E.EUNSTABLE
        with pytest.raises(E.EulbfsError):
            s.step(1)
    finally:
        s.close()


def test_supersonic_state_is_reported():
    # |u| = 0.8 > c_s = 1/sqrt(3): outside the low-Mach range of the flux reconstruction
    pr, st = PB.conductive_freezing()
    s = E.Solver(pr, st)
    try:
        w6 = s.conserved()
        w6[2] = 0.8 / 3.0  # rho c_s^2 u with rho = 1
        s.set_conserved(w6)
        with pytest.raises(E.EulbfsError) as ei:
            s.run(1)
        assert ei.value.code == E.EUNSTABLE
        assert "sound speed" in str(ei.value)
    finally:
        s.close()


def test_conductive_freezing_neumann_on_gpu():
    """The full 20 000-step run of Sec. 3.1 (one-phase) on the GPU: the front
    is within 0.5 cell of 2 k sqrt(alpha t) (k(0.1) = 0.2200163)."""
    import analytic as A

    pr, st = PB.conductive_freezing()
    s = E.Solver(pr, st)
    try:
        s.run(20000)
        d = s.diagnostics()
    finally:
        s.close()
    x_front = d["solid"] / (pr.ny * pr.dx)
    assert abs(x_front - A.neumann_front(0.1, 0.4, 20000 * pr.dt)) < 0.5


@pytest.mark.parametrize("ratio,c_source", [(0.8, 0), (1.2, 0), (0.8, 1)])
def test_full_freezing_height_on_gpu(oracle, ratio, c_source):
    """Sec. 3.2 run to full freezing (12 000 steps) on the GPU, expanding and
    contracting: the same state as the oracle to 1e-10 and the final solid height
    H_0 rho_l/rho_s within 0.05 cell (with the C-weighted reading of Eq. 40, the
    closed form (H_0 - (1 - r) xi/4) / r of that reading)."""
    import analytic as A

    H0 = 12.0
    pr, st = PB.stefan_full_freezing(ratio, H0=H0, ny=4, c_source=c_source)  # the library needs ny >= 4
    w6, _, d = _parity_run(oracle, pr, st, 12000)
    H_f = d["solid"] / (pr.ny * pr.dx)
    want = H0 / ratio if c_source == 0 else A.stefan_full_freezing_height_c_weighted(H0, ratio, pr.xi)
    assert abs(H_f - want) < 0.05


def test_two_phase_neumann_on_gpu(oracle):
    """Sec. 3.1 with its printed parameters (liquid at T_0 = 1, L = 250) for 8000
    steps on the GPU: the oracle's state to 1e-10 and the front within 0.1 cell of
    the two-phase Neumann front (Eq. 60 with erfc)."""
    import analytic as A

    pr, st = PB.conductive_freezing(nx=128, ny=4, ste=1.0 / 250.0)
    walls = dict(pr.walls)
    walls["x+"] = PB.Wall(PB.NOSLIP, PB.DIRICHLET, 1.0)
    pr = pr.replace(walls=walls)
    st.T[:] = 1.0
    _, _, d = _parity_run(oracle, pr, st, 8000)
    k = A.neumann_two_phase_k(1.0 / 250.0, 1.0 / 250.0, 0.4, 0.4)
    assert abs(d["solid"] / pr.ny - 2.0 * k * (0.4 * 8000 * pr.dt) ** 0.5) < 0.1


def test_solvers_on_concurrent_streams_are_independent():
    """Two solvers on two created streams, their steps enqueued alternately
    so that their launches overlap on the device, end bitwise where each ends
    alone: handles share no device state."""
    import torch

    cases = [PB.static_droplet(n=128, R=32, sigma=0.015625), PB.film_freezing(n=96)]
    alone = []
    for pr, st in cases:
        s = E.Solver(pr, st, kernel=E.KERNEL_AUTO, stream=torch.cuda.Stream())
        try:
            s.run(240)
            alone.append(s.conserved())
        finally:
            s.close()
    solvers = [E.Solver(pr, st, kernel=E.KERNEL_AUTO, stream=torch.cuda.Stream()) for pr, st in cases]
    try:
        for _ in range(30):
            for s in solvers:
                s.step(8)
        for s, ref in zip(solvers, alone):
            assert np.array_equal(s.conserved(), ref)
    finally:
        for s in solvers:
            s.close()
