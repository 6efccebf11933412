"""Problem descriptions and seeded synthetic initial states.

This module holds no arithmetic of the solver: it states a problem (grid,
material constants of Eq. (7), boundary conditions, the interface profiles of
Eqs. (61)-(62)) and produces the initial primitive fields (T, F_l, C, u, v, p)
as float64 planes of shape (ny, nx), row-major with x fastest.  The GPU
library and the CPU oracle each turn these into the conserved vector of
Eq. (49) with their own code.

Lattice units: the cell size is 1 unless ``dx`` says otherwise, the streaming
step ``delta_t`` is dx/2 (the largest value that keeps the surrounding points
of Eq. (54) inside the two cells sharing the face) and the update step ``dt``
is fixed for a run (Sec. 2.4, text after Eq. 58).

The configurations follow the paper's benchmark problems (Sec. 3.1-3.5) in
nondimensional form: melting temperature 0, cold wall -1, C_p = 1,
L = C_p (T_m - T_w) / Ste (Stefan number as defined in Sec. 3.2), liquid
density 1, interface width xi = 4 cells (Eq. 61), Q_g = 1, M_c = 0.1.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import Dict, Optional, Tuple

import numpy as np

NOSLIP, FREESLIP, OUTLET = 0, 1, 2
ADIABATIC, DIRICHLET = 0, 1
SIDES = ("x-", "x+", "y-", "y+")


@dataclass
class Wall:
    """One non-periodic side: flow rule, heat rule, wall temperature, contact
    angle and an optional hysteresis window [theta_rec, theta_adv] (0, 0: none)."""

    flow: int = NOSLIP
    heat: int = ADIABATIC
    T_w: float = 0.0
    theta_deg: float = 90.0
    theta_adv: float = 0.0
    theta_rec: float = 0.0


@dataclass
class Problem:
    nx: int
    ny: int
    dx: float = 1.0
    lattice_hg: int = 9
    delta_t: float = 0.5
    dt: float = 0.5
    # (solid, liquid, gas) for Eq. (7)
    rho: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    mu: Tuple[float, float, float] = (0.01, 0.01, 0.01)
    lam: Tuple[float, float, float] = (0.4, 0.4, 0.4)
    cp: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    latent: float = 10.0
    T_s: float = 0.0
    T_l: float = 0.0
    sigma: float = 0.0
    xi: float = 4.0
    mobility: float = 0.1
    Qg: float = 1.0
    gx: float = 0.0
    gy: float = 0.0
    surf_model: int = 0
    # C source of Eq. (40): 0: (1 - rho_s/rho_l) dF_s/dt with the cell's solid fraction
    # F_s = C (1 - F_l); 1: the printed factor C applied to that rate as well
    c_source: int = 0
    periodic_x: bool = False
    periodic_y: bool = False
    walls: Dict[str, Wall] = field(default_factory=dict)
    precision: int = 0  # 0: FP64; 1: FP32 fields and fluxes with FP64 enthalpy
    # stretched mesh: nx column widths and ny row heights (None: uniform dx)
    x_width: Optional[np.ndarray] = None
    y_width: Optional[np.ndarray] = None

    def wall(self, side: str) -> Optional[Wall]:
        periodic = self.periodic_x if side[0] == "x" else self.periodic_y
        if periodic:
            return None
        return self.walls.get(side, Wall())

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)

    @property
    def cells(self) -> int:
        return self.nx * self.ny


@dataclass
class InitialState:
    """Primitive initial fields, each float64 of shape (ny, nx)."""

    T: np.ndarray
    Fl: np.ndarray
    C: np.ndarray
    u: np.ndarray
    v: np.ndarray
    p: np.ndarray
    # the closed-form description these fields were built from, if any (the
    # library can build the same fields on the device from it)
    shape: Optional["Shape"] = None

    def planes(self):
        return [np.ascontiguousarray(a, dtype=np.float64) for a in (self.T, self.Fl, self.C, self.u, self.v, self.p)]


def widths(pr: Problem):
    """Column widths and row heights, (nx,) and (ny,) float64."""
    wx = np.full(pr.nx, pr.dx) if pr.x_width is None else np.asarray(pr.x_width, dtype=np.float64)
    wy = np.full(pr.ny, pr.dx) if pr.y_width is None else np.asarray(pr.y_width, dtype=np.float64)
    return wx, wy


def centres_1d(w: np.ndarray) -> np.ndarray:
    """Cell centres of a row of cells with widths w, the first face at 0."""
    return np.cumsum(w) - 0.5 * w


def cell_centres(pr: Problem):
    wx, wy = widths(pr)
    return np.meshgrid(centres_1d(wx), centres_1d(wy))  # (ny, nx) each


def graded_widths(n: int, w0: float, growth: float, w_max: float, both_ends: bool = False) -> np.ndarray:
    """n widths growing geometrically by `growth` from w0 at the start (and at
    the end too with both_ends) up to w_max: a mesh refined towards a wall."""
    i = np.arange(n, dtype=np.float64)
    d = np.minimum(i, n - 1 - i) if both_ends else i
    return np.minimum(w0 * growth ** d, w_max)


def layer_profile(coord: np.ndarray, H0: float, xi: float) -> np.ndarray:
    """Eq. (61): condensed phase below coord = H0."""
    return 0.5 * (1.0 + np.tanh(2.0 * (H0 - coord) / xi))


def droplet_profile(X, Y, x0, y0, R, xi):
    """Eq. (62) with the distance to the centre (the printed form lacks the square root)."""
    r = np.sqrt((X - x0) ** 2 + (Y - y0) ** 2)
    return 0.5 * (1.0 + np.tanh(2.0 * (R - r) / xi))


def uniform_state(pr: Problem, T0: float = 0.0, Fl0: float = 1.0, C0: float = 1.0) -> InitialState:
    shape = (pr.ny, pr.nx)
    return InitialState(
        T=np.full(shape, T0), Fl=np.full(shape, Fl0), C=np.full(shape, C0),
        u=np.zeros(shape), v=np.zeros(shape), p=np.zeros(shape),
    )


def splitmix_uniform(seed: int, n: np.ndarray) -> np.ndarray:
    """Outputs number n of the splitmix64 generator with state `seed` (Steele,
    Lea and Flood, OOPSLA 2014: the state advances by 0x9E3779B97F4A7C15 and
    each output is its mix), the top 53 bits as numbers uniform in [-1, 1)."""
    with np.errstate(over="ignore"):  # arithmetic modulo 2^64
        z = np.uint64(seed) + np.asarray(n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0


PROFILE_UNIFORM, PROFILE_LAYER, PROFILE_DROPLET = 0, 1, 2


@dataclasses.dataclass
class Shape:
    """A closed-form initial state: the condensed phase uniform (c0), below a
    flat interface (Eq. 61, at h0 across x or y) or inside a circle (Eq. 62,
    centre (x0, y0), radius r0); T = t_in where C > 1/2, else t_out, plus
    t_amp times splitmix_uniform(seed, j nx + i + 1); F_l = fl0; velocity
    (u_in, v_in) C; p = 0."""

    profile: int = PROFILE_UNIFORM
    axis: int = 0
    c0: float = 1.0
    h0: float = 0.0
    x0: float = 0.0
    y0: float = 0.0
    r0: float = 0.0
    t_out: float = 0.0
    t_in: float = 0.0
    t_amp: float = 0.0
    seed: int = 0
    fl0: float = 1.0
    u_in: float = 0.0
    v_in: float = 0.0

    def state(self, pr: "Problem") -> InitialState:
        """The fields on the problem's mesh (the host-side twin of the
        library's analytic initialisation)."""
        X, Y = cell_centres(pr)
        if self.profile == PROFILE_LAYER:
            C = layer_profile(X if self.axis == 0 else Y, self.h0, pr.xi)
        elif self.profile == PROFILE_DROPLET:
            C = droplet_profile(X, Y, self.x0, self.y0, self.r0, pr.xi)
        else:
            C = np.full((pr.ny, pr.nx), float(self.c0))
        T = np.where(C > 0.5, float(self.t_in), float(self.t_out))
        if self.t_amp != 0.0:
            n = np.arange(1, pr.nx * pr.ny + 1, dtype=np.uint64).reshape(pr.ny, pr.nx)
            T = T + self.t_amp * splitmix_uniform(self.seed, n)
        zero = np.zeros((pr.ny, pr.nx))
        u = self.u_in * C if self.u_in != 0.0 else zero.copy()
        v = self.v_in * C if self.v_in != 0.0 else zero.copy()
        return InitialState(T=T, Fl=np.full((pr.ny, pr.nx), float(self.fl0)), C=C, u=u, v=v, p=zero.copy(),
                            shape=self)


def seeded_fields(pr: Problem, seed: int, amp: float = 1.0) -> InitialState:
    """Smooth random primitive fields for parity checks (not a physical state)."""
    rng = np.random.default_rng(seed)
    X, Y = cell_centres(pr)
    wx, wy = widths(pr)
    Lx = pr.nx * pr.dx if pr.x_width is None else float(wx.sum())
    Ly = pr.ny * pr.dx if pr.y_width is None else float(wy.sum())

    def smooth(a0, a1):
        out = np.full(X.shape, a0)
        for _ in range(3):
            kx, ky = rng.integers(1, 3, size=2)
            ph = rng.uniform(0, 2 * np.pi, size=2)
            out = out + a1 * rng.uniform(-1, 1) * np.sin(2 * np.pi * kx * X / Lx + ph[0]) * np.cos(
                2 * np.pi * ky * Y / Ly + ph[1])
        return out

    C = np.clip(smooth(0.5, 0.35 * amp) + 0.02 * amp * rng.uniform(-1, 1, X.shape), -0.02, 1.02)
    T = smooth(0.0, 0.6 * amp) + 0.05 * amp * rng.uniform(-1, 1, X.shape)
    Fl = np.clip(smooth(0.5, 0.6), 0.0, 1.0)
    u = smooth(0.0, 0.03 * amp)
    v = smooth(0.0, 0.03 * amp)
    p = smooth(0.0, 0.01 * amp)
    return InitialState(T=T, Fl=Fl, C=C, u=u, v=v, p=p)


# ---------------------------------------------------------------------------
# Benchmark configurations (nondimensional, lattice units)
# ---------------------------------------------------------------------------
RHO_G = 1e-3  # gas / liquid density ratio 1/1000


def _gas_lambda(lam_l: float, rho_g: float) -> float:
    # gas thermal diffusivity equal to the liquid's (the paper gives no gas data)
    return lam_l * rho_g


def _gas_mu(mu_l: float, rho_g: float) -> float:
    # gas kinematic viscosity equal to the liquid's; a gas at 1/1000 of the
    # liquid density with 1/100 of its viscosity would need a smaller update step
    return mu_l * rho_g


def ch_mobility(sigma: float) -> float:
    """Cahn-Hilliard mobility M_c: the rate at which the interface profile is
    restored scales with M_c sigma / xi^2, so a weak surface tension (high
    Weber number) gets a larger mobility, M_c sigma >= 1e-3, between 0.1 and
    2.5 (tau_g - 1/2 = M_c / (Q_g delta_t) <= 5)."""
    return min(2.5, max(0.1, 1e-3 / sigma)) if sigma > 0 else 0.1


def conductive_freezing(nx: int = 128, ny: int = 4, ste: float = 0.1, **kw) -> Tuple[Problem, InitialState]:
    """Sec. 3.1 in its one-phase form: liquid at the melting point, cold left wall
    at -1, adiabatic right wall, periodic in y, no flow, C = 1 everywhere."""
    pr = Problem(
        nx=nx, ny=ny, rho=(1.0, 1.0, 1.0), mu=(0.01, 0.01, 0.01), lam=(0.4, 0.4, 0.4),
        cp=(1.0, 1.0, 1.0), latent=1.0 / ste, periodic_y=True,
        walls={"x-": Wall(NOSLIP, DIRICHLET, -1.0), "x+": Wall(NOSLIP, ADIABATIC)},
    ).replace(**kw)
    return pr, Shape().state(pr)


def three_phase_stefan(nx: int = 256, ny: int = 8, H0: float = 128.0, ratio: float = 0.9,
                       ste: float = 0.1, **kw) -> Tuple[Problem, InitialState]:
    """Sec. 3.2 laid along x: cold wall at x = 0, liquid 0 < x < H0, gas beyond."""
    rho_g = RHO_G
    pr = Problem(
        nx=nx, ny=ny, rho=(ratio, 1.0, rho_g), mu=(0.01, 0.01, 1e-4),
        lam=(0.4, 0.4, _gas_lambda(0.4, rho_g)), cp=(1.0, 1.0, 1.0), latent=1.0 / ste,
        sigma=0.01, periodic_y=True,
        walls={"x-": Wall(NOSLIP, DIRICHLET, -1.0), "x+": Wall(NOSLIP, ADIABATIC)},
    ).replace(**kw)
    return pr, Shape(profile=PROFILE_LAYER, axis=0, h0=H0).state(pr)


def stefan_full_freezing(ratio: float, nx: int = 32, ny: int = 1, H0: float = 12.0, ste: float = 0.25,
                         T0: float = 0.1, T_w: float = -2.0, latent: float = 250.0, rho_g: float = 0.01,
                         **kw) -> Tuple[Problem, InitialState]:
    """Sec. 3.2 with its printed temperatures and latent heat (T_0 = 0.1, T_w = -2,
    L = 250, T_m = 0, C_p,s = C_p,l, lambda_s = lambda_l), C_p taken from the Stefan
    number Ste = C_p (T_m - T_w) / L, run until the whole liquid column is frozen.
    The conductivity 0.4 C_p keeps the liquid diffusivity at 0.4 whatever Ste is
    (the paper prints only the ratio).  The paper gives no gas data; the gas is
    1/100 of the liquid density here (at 1/1000 the contracting cases,
    rho_s/rho_l >= 1.15, go unstable once the freezing front enters the gas side
    of the diffuse interface) with the liquid's thermal diffusivity and ten times
    its kinematic viscosity."""
    cp = ste * latent / (0.0 - T_w)
    pr = Problem(
        nx=nx, ny=ny, rho=(ratio, 1.0, rho_g), mu=(0.01, 0.01, 0.1 * rho_g),
        lam=(0.4 * cp, 0.4 * cp, 0.4 * cp * rho_g), cp=(cp, cp, cp), latent=latent,
        sigma=0.01, periodic_y=True,
        walls={"x-": Wall(NOSLIP, DIRICHLET, T_w), "x+": Wall(NOSLIP, ADIABATIC)},
    ).replace(**kw)
    return pr, Shape(profile=PROFILE_LAYER, axis=0, h0=H0, t_out=T0, t_in=T0).state(pr)


def film_freezing(n: int = 256, height: float = 0.3, ratio: float = 0.917, ste: float = 0.05,
                  bond: float = 1.0, seed: int = 0, amp: float = 1e-3, **kw) -> Tuple[Problem, InitialState]:
    """Sec. 3.3: film of height 0.3 n on a cold bottom wall in a closed box."""
    rho_g = RHO_G
    H0 = height * n
    sigma = 0.01
    g = bond * sigma / (1.0 * H0 * H0)
    pr = Problem(
        nx=n, ny=n, rho=(ratio, 1.0, rho_g), mu=(0.05, 0.05, _gas_mu(0.05, rho_g)),
        lam=(0.4, 0.4, _gas_lambda(0.4, rho_g)), cp=(1.0, 1.0, 1.0), latent=1.0 / ste,
        sigma=sigma, gy=-g,
        walls={"x-": Wall(), "x+": Wall(), "y-": Wall(NOSLIP, DIRICHLET, -1.0), "y+": Wall()},
    ).replace(**kw)
    return pr, Shape(profile=PROFILE_LAYER, axis=1, h0=H0, t_amp=amp, seed=seed).state(pr)


def static_droplet(n: int = 512, R: float = 128.0, theta_deg: float = 90.0, ratio: float = 0.917,
                   ste: float = 0.1, ca: float = 0.01, **kw) -> Tuple[Problem, InitialState]:
    """Sec. 3.4: droplet resting on a cold bottom wall (a half disc for 90 deg)."""
    rho_g = RHO_G
    lam_l = 0.4
    u_ref = lam_l / (1.0 * 1.0) / R  # thermal velocity alpha_l / R
    mu_l = 0.05
    sigma = mu_l * u_ref / ca
    pr = Problem(
        nx=n, ny=n, rho=(ratio, 1.0, rho_g), mu=(mu_l, mu_l, _gas_mu(mu_l, rho_g)),
        lam=(lam_l, lam_l, _gas_lambda(lam_l, rho_g)), cp=(1.0, 1.0, 1.0), latent=1.0 / ste,
        sigma=sigma,
        walls={"x-": Wall(), "x+": Wall(), "y-": Wall(NOSLIP, DIRICHLET, -1.0, theta_deg), "y+": Wall()},
    ).replace(**kw)
    x0 = 0.5 * pr.nx * pr.dx
    # circular cap of the same area as a half disc of radius R, meeting the wall at theta
    th = math.radians(theta_deg)
    Rc = R * math.sqrt((math.pi / 2.0) / (th - math.sin(th) * math.cos(th)))
    y0 = -Rc * math.cos(th)
    return pr, Shape(profile=PROFILE_DROPLET, x0=x0, y0=y0, r0=Rc).state(pr)


# Table 3 of the paper (SI units): liquid and solid properties of the two fluids
# of Sec. 3.4, the wall temperature and the melting point.
TABLE3 = {
    "water": {"rho": (917.0, 999.0), "cp": (2100.0, 4220.0), "lam": (2.16, 0.581), "latent": 333400.0,
              "T_m": 0.0, "T_w": -10.0},
    "hexadecane": {"rho": (833.0, 774.0), "cp": (1800.0, 2310.0), "lam": (0.15, 0.15), "latent": 230000.0,
                   "T_m": 18.0, "T_w": 15.0},
}


# Table 1 (Sec. 3.3): water, (liquid, solid), SI units
TABLE1 = {"rho": (1000.0, 917.0), "cp": (4210.0, 2030.0), "lam": (0.56, 2.20), "latent": 334000.0,
          "T_m": 0.0, "T_w": -20.0, "T_0": 20.0}


def film_table1(ratio: float = 0.917, nx: int = 200, ny: int = 400, H0: float = 100.0, alpha_l: float = 0.05,
                **kw) -> Tuple[Problem, InitialState]:
    """Sec. 3.3: a water film (Table 1) in a 2-D container on the paper's 200 x 400
    grid, cooled from the left and bottom walls (T_w = -20 C), liquid and gas at
    T_0 = 20 C, a symmetry plane on the right (free slip, adiabatic) and an outlet
    at the top (adiabatic); no-flux phase field on every wall.  Lattice map as for
    the Table 3 fluids: rho_l = C_p,l = 1, the solid keeps the printed C_p and
    lambda ratios and rho_s/rho_l = `ratio` (Table 2 runs 1 and 0.917), T_m - T_w
    -> 1, L -> L / (C_p,l (T_m - T_w)), alpha_l = 0.05, mu_l = 0.05.  The paper
    prints no film height (H0 cells here), no surface tension in lattice units
    (0.01, as the 256 x 256 film) and no gas data (the gas of the other
    configurations)."""
    m = TABLE1
    cpl, cps = m["cp"]
    laml, lams = m["lam"]
    dT = m["T_m"] - m["T_w"]
    lam_l = alpha_l
    lam_s = lam_l * lams / laml
    mu_l = 0.05
    rho_g = RHO_G
    pr = Problem(
        nx=nx, ny=ny, rho=(ratio, 1.0, rho_g), mu=(mu_l, mu_l, _gas_mu(mu_l, rho_g)),
        lam=(lam_s, lam_l, _gas_lambda(lam_l, rho_g)), cp=(cps / cpl, 1.0, 1.0), latent=m["latent"] / (cpl * dT),
        sigma=0.01,
        walls={"x-": Wall(NOSLIP, DIRICHLET, -1.0), "y-": Wall(NOSLIP, DIRICHLET, -1.0),
               "x+": Wall(FREESLIP, ADIABATIC), "y+": Wall(OUTLET, ADIABATIC)},
    ).replace(**kw)
    T0 = (m["T_0"] - m["T_m"]) / dT
    return pr, Shape(profile=PROFILE_LAYER, axis=1, h0=H0, t_out=T0, t_in=T0).state(pr)


def table3_droplet(fluid: str, theta_deg: float, ratio: float = None, nx: int = 400, ny: int = 200,
                   R: float = 50.0, alpha_l: float = 0.05, **kw) -> Tuple[Problem, InitialState]:
    """Sec. 3.4 volume-change runs (Figs. 11-12): a sessile droplet of one of the
    Table 3 fluids on a cold wall at contact angle theta, on the paper's 400 x 200
    grid.  Lattice map: the liquid is rho_l = 1, C_p,l = 1, alpha_l = alpha_l; the
    solid keeps the Table 3 ratios rho_s/rho_l (or `ratio`), C_p,s/C_p,l and
    lambda_s/lambda_l; T_m - T_w maps to 1 and L to L / (C_p,l (T_m - T_w)).  The
    droplet starts at T_m (the pre-nucleation state).  The paper gives no gas data
    and no lattice viscosity or surface tension: the gas follows the other
    configurations (1/1000 of the liquid density, the liquid's diffusivity and
    kinematic viscosity); mu_l = 0.05 and sigma from Ca = 0.01 on the thermal
    velocity alpha_l / R, as for the 512 x 512 droplet (with mu_l = alpha_l / 8 the
    light gas at a 135 deg contact line goes unstable within 300 steps)."""
    m = TABLE3[fluid]
    rs, rl = m["rho"]
    r = rs / rl if ratio is None else ratio
    cps, cpl = m["cp"]
    lams, laml = m["lam"]
    cp_s = cps / cpl
    lam_l = alpha_l * 1.0 * 1.0
    lam_s = lam_l * lams / laml
    latent = m["latent"] / (cpl * (m["T_m"] - m["T_w"]))
    mu_l = 0.05
    rho_g = RHO_G
    sigma = mu_l * (alpha_l / R) / 0.01
    pr = Problem(
        nx=nx, ny=ny, rho=(r, 1.0, rho_g), mu=(mu_l, mu_l, _gas_mu(mu_l, rho_g)),
        lam=(lam_s, lam_l, _gas_lambda(lam_l, rho_g)), cp=(cp_s, 1.0, 1.0), latent=latent,
        sigma=sigma,
        walls={"x-": Wall(), "x+": Wall(), "y-": Wall(NOSLIP, DIRICHLET, -1.0, theta_deg), "y+": Wall()},
    ).replace(**kw)
    th = math.radians(theta_deg)
    Rc = R * math.sqrt((math.pi / 2.0) / (th - math.sin(th) * math.cos(th)))
    return pr, Shape(profile=PROFILE_DROPLET, x0=0.5 * pr.nx * pr.dx, y0=-Rc * math.cos(th), r0=Rc).state(pr)


def impact_droplet(n: int = 256, we: float = 50.0, re: float = 500.0, U: float = 0.05,
                   ratio: float = 0.917, ste: float = 0.1, supercool: float = 0.5,
                   theta_deg: float = 90.0, **kw) -> Tuple[Problem, InitialState]:
    """Sec. 3.5: droplet of diameter n/4 moving down onto a cold wall; the
    surface tension acts on the unfrozen part only (surf_model 1)."""
    rho_g = RHO_G
    D = n / 4.0
    sigma = 1.0 * U * U * D / we
    mu_l = 1.0 * U * D / re
    lam_l = 0.4
    pr = Problem(
        nx=n, ny=n, rho=(ratio, 1.0, rho_g), mu=(mu_l, mu_l, _gas_mu(mu_l, rho_g)),
        lam=(lam_l, lam_l, _gas_lambda(lam_l, rho_g)), cp=(1.0, 1.0, 1.0), latent=1.0 / ste,
        sigma=sigma, mobility=ch_mobility(sigma), surf_model=1,
        walls={"x-": Wall(), "x+": Wall(), "y-": Wall(NOSLIP, DIRICHLET, -1.0, theta_deg), "y+": Wall()},
    ).replace(**kw)
    x0 = 0.5 * pr.nx * pr.dx
    y0 = 0.5 * D + 2.0 * pr.xi
    return pr, Shape(profile=PROFILE_DROPLET, x0=x0, y0=y0, r0=0.5 * D, t_in=-supercool, v_in=-U).state(pr)


# Sec. 3.5 impact cases (SI units): the droplet, the impact speed, the
# initial and wall temperatures and the contact angles of case (a) and (b)
IMPACT_CASES = {
    "a": {"D": 2.84e-3, "U": 0.7, "T_0": -5.0, "T_w": -30.0, "theta_adv": 100.0, "theta_rec": 39.0, "theta_eq": 82.0},
    "b": {"D": 2.62e-3, "U": 0.44, "T_0": 25.0, "T_w": -30.0, "theta_adv": 105.0, "theta_rec": 70.0, "theta_eq": 70.0},
}
# the gas: air at its ratios to the Table 1 water (viscosity 1.8e-5 Pa s,
# conductivity 0.026 W/(m K), heat capacity 1005 J/(kg K); the paper gives no
# gas data), at 1/1000 of the liquid density
AIR = {"mu": 0.0106, "lam": 0.046, "cp": 0.239}


def impact_sec35(case: str = "b", T_w: float = None, D0: float = 100.0, U: float = 0.05, nx: int = 400,
                 ny: int = 200, **kw) -> Tuple[Problem, InitialState]:
    """Sec. 3.5: a water droplet (Table 1 properties) of diameter D0 cells
    moving down at U onto a cold no-slip wall with contact-angle hysteresis,
    on the paper's 400 x 200 grid, walls adiabatic elsewhere, the surface force
    on the unfrozen part only.  Lattice map: rho_l = C_p,l = 1, T_m - T_w -> 1;
    Re = rho U D/mu, We = rho U^2 D/sigma and Pr = mu C_p/lambda of the case set
    the lattice viscosity, surface tension and conductivity; Ste = C_p (T_m -
    T_w)/L; the solid keeps the Table 1 ratios; the gas is AIR.  T_w (deg C)
    overrides the case's wall temperature (Table 7 varies it)."""
    c = IMPACT_CASES[case]
    m = TABLE1
    rho_l, rho_s = m["rho"]
    cp_l, cp_s = m["cp"]
    lam_l, lam_s = m["lam"]
    mu_l, sigma_l = 0.0017, 0.076  # Table 1
    Tw = c["T_w"] if T_w is None else T_w
    dT = m["T_m"] - Tw
    Re = rho_l * c["U"] * c["D"] / mu_l
    We = rho_l * c["U"] ** 2 * c["D"] / sigma_l
    Pr = mu_l * cp_l / lam_l
    nu = U * D0 / Re
    sigma = U * U * D0 / We
    lam = nu / Pr
    pr = Problem(
        nx=nx, ny=ny, rho=(rho_s / rho_l, 1.0, RHO_G), mu=(nu, nu, AIR["mu"] * nu),
        lam=(lam * lam_s / lam_l, lam, AIR["lam"] * lam), cp=(cp_s / cp_l, 1.0, AIR["cp"]),
        latent=m["latent"] / (cp_l * dT), sigma=sigma, mobility=ch_mobility(sigma), surf_model=1,
        walls={"x-": Wall(), "x+": Wall(), "y+": Wall(),
               "y-": Wall(NOSLIP, DIRICHLET, -1.0, c["theta_eq"], c["theta_adv"], c["theta_rec"])},
    ).replace(**kw)
    T0 = (c["T_0"] - m["T_m"]) / dT
    sh = Shape(profile=PROFILE_DROPLET, x0=0.5 * pr.nx * pr.dx, y0=0.5 * D0 + 2.0 * pr.xi, r0=0.5 * D0,
               t_in=T0, t_out=T0, v_in=-U)
    return pr, sh.state(pr)


def impact_time(case: str, t_seconds: float, D0: float = 100.0, U: float = 0.05) -> float:
    """Lattice time of a physical time of a Sec. 3.5 case (t U / D in both)."""
    c = IMPACT_CASES[case]
    return t_seconds * c["U"] / c["D"] * D0 / U


CONFIGS = {
    "C1": lambda: conductive_freezing(),
    "C2": lambda: three_phase_stefan(),
    "C3": lambda: film_freezing(),
    "C4": lambda: static_droplet(),
}
