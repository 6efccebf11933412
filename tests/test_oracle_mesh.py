"""Pins of the oracle on stretched tensor-product meshes (Eq. 52 with general
cell volumes and face areas; the paper runs uniform meshes only).

Each test checks the oracle against the mathematics, not against itself:
derivatives exact on parabolas, the extrapolation of Eq. (54) from each cell
centre to its own face distance, linear profiles that are steady states
whatever the spacing, conservation of the phase field through the volume and
face weights, mirror symmetry, the wetting ghosts as the linear continuation
of a profile through the wall, and the two-phase Neumann solution of Sec. 3.1
on a mesh refined towards the cold wall.  The comments name the mistake each
one is there to catch.
"""
import math
import os

import numpy as np
import pytest

import analytic as A
from paper_2507_03366_amd import problems as PB


def _golden(name):
    """key = values lines of a fixture under tests/golden (numbers only)."""
    out = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                key, vals = line.split("=")
                out[key.strip()] = [float(x) for x in vals.split()]
    return out


def _widths(n, seed, lo=0.6, hi=1.4):
    return np.random.default_rng(seed).uniform(lo, hi, size=n)


def _liquid(pr, T):
    """All-liquid state (C = 1, F_l = 1) at rest with temperature T (ny, nx)."""
    st = PB.uniform_state(pr)
    st.T = np.array(T, dtype=np.float64)
    return st


def test_chemical_potential_exact_on_a_parabola(oracle):
    """mu_c = 2 beta C (C-1)(2C-1) - kappa lap C with lap C of a parabola
    C = c0 + a (x - x0)^2 + b (y - y0)^2 equal to 2 (a + b) at every cell whose
    stencil is interior, whatever the widths.  Catches a Laplacian divided by
    the cell width instead of the mean centre distance, or neighbours' centre
    distances taken from the wrong side."""
    nx, ny = 14, 12
    pr = PB.Problem(nx=nx, ny=ny, sigma=0.02, x_width=_widths(nx, 1), y_width=_widths(ny, 2), delta_t=0.3)
    X, Y = PB.cell_centres(pr)
    a, b = 2e-4, -1.5e-4
    C = 0.5 + a * (X - 6.0) ** 2 + b * (Y - 5.0) ** 2
    st = PB.uniform_state(pr, T0=1.0)
    st.C = C
    W = oracle.init(pr, st)
    muc = oracle.primitives(pr, W)[6]
    beta, kappa = 12.0 * pr.sigma / pr.xi, 1.5 * pr.xi * pr.sigma
    exact = 2.0 * beta * C * (C - 1.0) * (2.0 * C - 1.0) - kappa * 2.0 * (a + b)
    inner = (slice(1, ny - 1), slice(1, nx - 1))
    np.testing.assert_allclose(muc[inner], exact[inner], rtol=0, atol=1e-13)


@pytest.mark.parametrize("lattice", [9, 5])
@pytest.mark.parametrize("axis", ["x", "y"])
def test_heat_flux_extrapolates_each_side_by_its_own_half_width(oracle, lattice, axis):
    """Liquid at rest, uniform properties, temperature varying along one axis.
    With u = 0 the enthalpy flux is k (A - B) with k fixed by lambda, rho and
    delta_t, A the value the upwind cell a extrapolates to x_f - delta_t and B
    the value cell b extrapolates to x_f + delta_t (Eq. 54).  k is read off a
    linear profile (exact extrapolation); for T = c0 + c1 s + c2 s^2 an exact
    centre derivative leaves A = T(x_f - delta_t) - c2 (w_a/2 - delta_t)^2 and
    B = T(x_f + delta_t) - c2 (w_b/2 - delta_t)^2 (Taylor).  Catches a centre
    derivative that is not exact on parabolas (the plain central difference over
    unequal spacings), the two half widths swapped or taken from one side, and a
    face placed at the mean of the two centres."""
    n, m = 16, 4
    w = _widths(n, 7)
    dt = 0.25
    kw = dict(lattice_hg=lattice, delta_t=dt, periodic_x=axis == "y", periodic_y=axis == "x",
              T_s=0.0, T_l=0.0, latent=1.0)
    if axis == "x":
        pr = PB.Problem(nx=n, ny=m, x_width=w, **kw)
    else:
        pr = PB.Problem(nx=m, ny=n, y_width=w, **kw)
    s = PB.centres_1d(w)
    faces = np.concatenate([[0.0], np.cumsum(w)])

    def fluxes(T1):
        T = np.broadcast_to(T1[None, :] if axis == "x" else T1[:, None], (pr.ny, pr.nx))
        W = oracle.init(pr, _liquid(pr, T))
        _, Fx, Fy = oracle.residual(pr, W)
        return Fx[0][0] if axis == "x" else Fy[0][:, 0]

    c0, c1 = 3.0, 0.05
    lin = fluxes(c0 + c1 * s)
    f = np.arange(3, n - 2)  # interior faces whose stencils stay inside
    k = lin[f] / (-2.0 * dt * c1)
    assert np.ptp(k) <= 1e-12 * abs(k).max()  # a linear profile: one k on every face
    k = k.mean()
    c2 = 4e-3
    T = lambda x: c0 + c1 * x + c2 * x * x
    quad = fluxes(T(s))
    ha, hb = 0.5 * w[f - 1], 0.5 * w[f]
    A_ = T(faces[f] - dt) - c2 * (ha - dt) ** 2
    B_ = T(faces[f] + dt) - c2 * (hb - dt) ** 2
    np.testing.assert_allclose(quad[f], k * (A_ - B_), rtol=1e-11, atol=0)


@pytest.mark.parametrize("lattice", [9, 5])
def test_linear_conduction_is_steady_between_dirichlet_walls(oracle, lattice):
    """A liquid slab between walls held at T = 1 and T = 2 with the exact
    linear profile on a stretched mesh is a steady state: every residual is zero
    to rounding, the wall cells included.  The Dirichlet ghost T_g = 2 T_w - T_m
    continues the line only if the ghost has the width of its mirror cell, so
    this catches ghost widths taken from the uniform spacing or from the wrong
    interior cell, and fluxes scaled by the wrong cell's width."""
    nx, ny = 18, 3
    w = _widths(nx, 11)
    L = w.sum()
    pr = PB.Problem(nx=nx, ny=ny, x_width=w, y_width=_widths(ny, 12), lattice_hg=lattice, delta_t=0.28,
                    T_s=0.0, T_l=0.0, latent=1.0, periodic_y=True,
                    walls={"x-": PB.Wall(PB.NOSLIP, PB.DIRICHLET, 1.0), "x+": PB.Wall(PB.NOSLIP, PB.DIRICHLET, 2.0)})
    X, _ = PB.cell_centres(pr)
    W = oracle.init(pr, _liquid(pr, 1.0 + X / L))
    R, Fx, _ = oracle.residual(pr, W)
    assert abs(Fx[0]).max() > 1e-4  # heat does flow
    np.testing.assert_allclose(R, 0.0, atol=1e-13)


def test_phase_field_conserved_on_a_stretched_box(oracle):
    """Flowing drop in a closed box with no-flux wetting walls and cells of
    unequal widths in both directions: sum C w_i h_j stays constant to rounding.
    Only volumes and face areas that match (Eq. 52: V = w_i h_j, S = h_j or w_i)
    telescope, so this catches a residual scaled by a neighbour's width, a face
    area taken along the wrong direction and a diagnostic volume with the two
    directions mixed up."""
    oracle.set_threads(8)
    n = 24
    pr = PB.Problem(nx=n, ny=n, rho=(1.0, 1.0, 0.1), mu=(0.05, 0.05, 0.005), lam=(0.4, 0.4, 0.04),
                    sigma=0.01, delta_t=0.3, dt=0.3, x_width=_widths(n, 21), y_width=_widths(n, 22, 0.7, 1.6),
                    walls={s: PB.Wall(heat=PB.DIRICHLET, T_w=-1.0, theta_deg=60.0) if s == "y-"
                           else PB.Wall(theta_deg=110.0) for s in PB.SIDES})
    X, Y = PB.cell_centres(pr)
    st = PB.uniform_state(pr)
    st.C = PB.droplet_profile(X, Y, 11.0, 9.0, 6.0, 4.0)
    st.u = 0.01 * st.C
    W0 = oracle.init(pr, st)
    W, _ = oracle.step(pr, W0, np.zeros((n, n)), 150)
    wx, wy = PB.widths(pr)
    V = wy[:, None] * wx[None, :]
    c0, c1 = (V * W0[4]).sum(), (V * W[4]).sum()
    assert abs(c1 - c0) <= 1e-12 * c0
    assert abs(oracle.diagnostics(pr, W)[1] - c1) <= 1e-12 * c0
    assert abs(W[4] - W0[4]).max() > 1e-3  # the drop did move


def test_mirror_symmetric_mesh_keeps_a_centred_drop_symmetric(oracle):
    """Mesh graded towards both x walls (mirror-symmetric), drop on the centre
    line, walls of one kind: C stays even and M_x odd under x -> -x to rounding.
    Catches the x+ wall reading its distances from the x- end and a face
    extrapolation that favours one side."""
    oracle.set_threads(8)
    nx, ny = 20, 16
    w = PB.graded_widths(nx, 0.6, 1.2, 1.4, both_ends=True)
    pr = PB.Problem(nx=nx, ny=ny, rho=(1.0, 1.0, 0.1), mu=(0.05, 0.05, 0.005), lam=(0.4, 0.4, 0.04),
                    sigma=0.01, delta_t=0.3, dt=0.3, x_width=w, gy=-1e-4,
                    walls={s: PB.Wall(theta_deg=70.0) for s in PB.SIDES})
    X, Y = PB.cell_centres(pr)
    st = PB.uniform_state(pr)
    st.C = PB.droplet_profile(X, Y, 0.5 * w.sum(), 4.0, 6.0, 4.0)
    W, _ = oracle.run(pr, st, 120)
    np.testing.assert_allclose(W[4], W[4][:, ::-1], atol=1e-11)
    np.testing.assert_allclose(W[2], -W[2][:, ::-1], atol=1e-11)
    assert abs(W[3]).max() > 1e-6  # something moves


@pytest.mark.parametrize("side", ["x-", "x+", "y-", "y+"])
def test_wetting_ghosts_continue_a_line_through_a_stretched_wall(oracle, side):
    """Ghost k mirrors interior cell k-1, whose centre lies s_k from the wall,
    so the ghost centre is 2 s_k from the mirror.  (1) Plain wall at theta:
    C_g - C_m = 2 s_k (4/xi) cos(theta) C_w (1 - C_w).  (2) Hysteresis window
    around the apparent angle of a profile linear along the normal: the
    apparent angle is read exactly from the parabola through three unequal
    centres, so the ghosts continue the line, C_g = C(-s_k).  (3) A window that
    excludes it pins the angle to the nearer bound.  Catches distances of the
    uniform mesh, a wall parabola through the wrong centres and the x+ or y+
    wall measured from the other end."""
    n, m = 10, 3
    w = _widths(n, 31, 0.5, 1.5)
    xside = side[0] == "x"
    kw = dict(delta_t=0.25, periodic_y=xside, periodic_x=not xside, sigma=0.01)
    pr = PB.Problem(nx=n, ny=m, x_width=w, **kw) if xside else PB.Problem(nx=m, ny=n, y_width=w, **kw)
    s = PB.centres_1d(w)
    d = s if side[1] == "-" else w.sum() - s  # distance of each centre from this wall
    order = np.argsort(d)  # interior cells outward from the wall
    c1 = 0.04
    C1d = 0.45 + c1 * d  # C grows linearly away from the wall

    def ghosts(theta, adv=0.0, rec=0.0):
        walls = {side: PB.Wall(theta_deg=theta, theta_adv=adv, theta_rec=rec)}
        for other in PB.SIDES:
            if other != side and other[0] == side[0]:
                walls[other] = PB.Wall()
        p = pr.replace(walls=walls)
        st = PB.uniform_state(p, T0=1.0)
        st.C = np.broadcast_to(C1d[None, :] if xside else C1d[:, None], (p.ny, p.nx)).copy()
        Wg = oracle.ghosts(p, oracle.init(p, st))[4]
        line = Wg[3, :] if xside else Wg[:, 3]  # one interior row (column) with its ghosts
        if side[1] == "-":
            g = line[2::-1]  # ghost layers k = 1, 2, 3 outward
        else:
            g = line[n + 3:]
        return g

    Cw = C1d[order[0]]
    mirror = C1d[order[:3]]
    dk = 2.0 * d[order[:3]]
    g = ghosts(50.0)
    np.testing.assert_allclose(g - mirror, dk * (4.0 / 4.0) * math.cos(math.radians(50.0)) * Cw * (1 - Cw),
                               rtol=1e-12)
    cos_app = -c1 / ((4.0 / 4.0) * Cw * (1 - Cw))
    th_app = math.degrees(math.acos(cos_app))
    g = ghosts(th_app, th_app + 10.0, th_app - 10.0)
    np.testing.assert_allclose(g, 0.45 - c1 * d[order[:3]], rtol=1e-12)
    g = ghosts(th_app + 20.0, th_app + 30.0, th_app + 15.0)  # window above the apparent angle
    cos_rec = math.cos(math.radians(th_app + 15.0))
    np.testing.assert_allclose(g - mirror, dk * cos_rec * Cw * (1 - Cw), rtol=1e-12)


def test_two_phase_neumann_on_a_mesh_refined_at_the_cold_wall(oracle):
    """Sec. 3.1 with its printed parameters on a mesh whose cells grow from 0.5
    at the cold wall to 1.5: the front (sum F_s w_i) is within 0.1 of
    2 k sqrt(alpha_s t) and the temperature away from the front within 0.01 of
    the two-phase Neumann profile (Eqs. 59-60 with erfc), as on the uniform
    mesh.  Catches any inconsistency between the stretched geometry and the
    physics of conduction with latent heat (wrong flux scaling, wrong ghost
    distance at the Dirichlet wall, a front integral without the widths)."""
    g = {k: v[0] for k, v in _golden("conductive_freezing_sec31.txt").items()}
    oracle.set_threads(1)
    w = PB.graded_widths(110, 0.5, 1.03, 1.5)
    nx, dt, steps = len(w), 0.25, 16000
    lam = g["alpha_s"] * g["rho_s"] * g["cp_s"]
    pr, st = PB.conductive_freezing(nx=nx, ny=1, ste=1.0 / g["L"])
    pr = pr.replace(walls={"x-": PB.Wall(PB.NOSLIP, PB.DIRICHLET, g["T_b"]),
                           "x+": PB.Wall(PB.NOSLIP, PB.DIRICHLET, g["T_0"])},
                    rho=(g["rho_s"], g["rho_l"], 1.0), cp=(g["cp_s"], g["cp_l"], 1.0), lam=(lam, lam, lam),
                    latent=g["L"], T_s=g["T_m"], T_l=g["T_m"], x_width=w, delta_t=0.25, dt=dt)
    st.T[:] = g["T_0"]
    W, _ = oracle.run(pr, st, steps)
    t = steps * dt
    st_s = g["cp_s"] * (g["T_m"] - g["T_b"]) / g["L"]
    st_l = g["cp_l"] * (g["T_0"] - g["T_m"]) / g["L"]
    k = A.neumann_two_phase_k(st_s, st_l, g["alpha_s"], g["alpha_l"])
    x_i = 2.0 * k * math.sqrt(g["alpha_s"] * t)
    front = oracle.diagnostics(pr, W)[3] / pr.dx
    assert abs(front - x_i) < 0.1
    X, _ = PB.cell_centres(pr)
    T = oracle.primitives(pr, W)[0][0]
    Tex = A.neumann_two_phase_T(X[0], t, k, g["T_b"], g["T_m"], g["T_0"], g["alpha_s"], g["alpha_l"])
    away = (np.abs(X[0] - x_i) > 1.5) & (X[0] < 0.5 * w.sum())
    assert np.abs(T - Tex)[away].max() < 0.01


def test_conduction_converges_at_second_order_on_a_smoothly_stretched_mesh(oracle):
    """Transient conduction from a wall held at 0.5 into liquid at 1 (no phase
    change) on meshes mapped by x = L (e^{b s} - 1) / (e^b - 1), b = 2 (the last
    cell 7.4 times the first), against T_w + (T_0 - T_w) erf(x / 2 sqrt(alpha t)):
    doubling the cells divides the largest error by at least 3 (measured 3.9,
    and 4.0 for the next doubling).  A cell volume taken from a neighbour, an
    O(h) relative error, drops it to first order (1.8); swapped half widths
    move the extrapolation only by O(h^2) on such a mesh and are left to the
    face-flux pin above."""
    oracle.set_threads(1)
    Lx, b, t_end, alpha = 40.0, 2.0, 12.0, 0.4
    errs = []
    for n in (40, 80):
        s = np.arange(n + 1) / n
        xf = Lx * (np.exp(b * s) - 1.0) / (math.exp(b) - 1.0)
        w = np.diff(xf)
        dt = 0.25 * w.min() ** 2 / alpha
        steps = int(round(t_end / dt))
        dt = t_end / steps
        pr = PB.Problem(nx=n, ny=1, x_width=w, delta_t=0.25 * w.min(), dt=dt, lam=(alpha, alpha, alpha),
                        T_s=0.0, T_l=0.0, latent=1.0, periodic_y=True,
                        walls={"x-": PB.Wall(PB.NOSLIP, PB.DIRICHLET, 0.5), "x+": PB.Wall(PB.NOSLIP, PB.ADIABATIC)})
        W, _ = oracle.run(pr, _liquid(pr, np.ones((1, n))), steps)
        T = oracle.primitives(pr, W)[0][0]
        x = PB.centres_1d(w)
        exact = np.array([0.5 + 0.5 * math.erf(xi / (2.0 * math.sqrt(alpha * t_end))) for xi in x])
        errs.append(np.abs(T - exact).max())
    assert errs[0] < 0.02
    assert errs[0] / errs[1] > 3.0, errs
