"""Closed forms and textbook solvers that pin the oracle (test infrastructure).

Nothing here calls the oracle or the GPU library.
"""
from __future__ import annotations

import math

import numpy as np


def neumann_k(ste: float) -> float:
    """One-phase Neumann constant: k exp(k^2) erf(k) = Ste / sqrt(pi).

    This is the transcendental relation of Sec. 3.1 (Eq. 60) with the liquid at
    the melting point (T_0 = T_m), where its second term vanishes; the front is
    X_i(t) = 2 k sqrt(alpha_s t).  Solved by bisection.
    """
    target = ste / math.sqrt(math.pi)
    lo, hi = 0.0, 3.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid * math.exp(mid * mid) * math.erf(mid) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def neumann_front(ste: float, alpha_s: float, t: float) -> float:
    return 2.0 * neumann_k(ste) * math.sqrt(alpha_s * t)


def neumann_two_phase_k(st_s: float, st_l: float, alpha_s: float, alpha_l: float) -> float:
    """Two-phase Neumann constant (Sec. 3.1, liquid above the melting point):

        St_s / (e^{k^2} erf k) - St_l sqrt(a_l/a_s) / (e^{k^2 a_s/a_l} erfc(k sqrt(a_s/a_l))) = k sqrt(pi)

    with St_s = C_p,s (T_m - T_b)/L and St_l = C_p,l (T_0 - T_m)/L.  This is the
    textbook balance of latent heat against the conductive fluxes of the two
    erf/erfc profiles; Eq. (60) prints erf where the liquid term needs erfc (the
    liquid profile decays to T_0 far from the front), and its form with erf has no
    root for the Sec. 3.1 parameters.  The left side falls monotonically in k
    from +inf, so bisection on (0, 3) finds the one root."""
    r = math.sqrt(alpha_s / alpha_l)

    def lhs(k):
        return (st_s / (math.exp(k * k) * math.erf(k))
                - st_l / r / (math.exp(k * k * r * r) * math.erfc(k * r)) - k * math.sqrt(math.pi))

    lo, hi = 1e-12, 3.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if lhs(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def neumann_two_phase_T(x: np.ndarray, t: float, k: float, T_b: float, T_m: float, T_0: float,
                        alpha_s: float, alpha_l: float) -> np.ndarray:
    """Temperature of the two-phase Neumann solution (Eq. 59 with the liquid
    branch written with erfc, which makes T = T_m at the front and T -> T_0 far
    from it; the printed liquid branch is neither).  Front at X_i = 2 k sqrt(a_s t)."""
    from scipy.special import erf, erfc

    xi = 2.0 * k * math.sqrt(alpha_s * t)
    sol = T_b + (T_m - T_b) * erf(x / (2.0 * np.sqrt(alpha_s * t))) / math.erf(k)
    kl = k * math.sqrt(alpha_s / alpha_l)
    liq = T_0 - (T_0 - T_m) * erfc(x / (2.0 * np.sqrt(alpha_l * t))) / math.erfc(kl)
    return np.where(x < xi, sol, liq)


def stefan_full_freezing_height_c_weighted(H0: float, ratio: float, xi: float) -> float:
    """Final solid height of the three-phase Stefan problem (Sec. 3.2) on a diffuse
    interface when the phase-field source of Eq. (40) is C (1 - rho_s/rho_l) dF_s/dt
    with the cell's solid fraction F_s = C (1 - F_l) (the c_source = 1 reading).

    Sharp interface: a frozen column of height H_f held the liquid column H_0 =
    (rho_s/rho_l) H_f, so H_f = H_0 rho_l / rho_s.  Under this reading, where the
    order parameter is below 1 a cell that freezes completely gains F_s = C, so it
    contributes C^2 (1 - r) instead of C (1 - r) to the condensed volume (r =
    rho_s/rho_l).  Summed over the column the deficit is (1 - r) D with D the
    integral of C (1 - C) across the interface, xi/4 for the tanh profile of Eq.
    (61).  Mass balance H_f = H_0 + (1 - r)(H_f - D) then gives
    H_f = (H_0 - (1 - r) xi/4) / r, which tends to H_0 / r as xi / H_0 -> 0.
    """
    return (H0 - (1.0 - ratio) * xi / 4.0) / ratio


def stefan_three_phase_interface(H0: float, ratio: float, ste: float, alpha_s: float, t: float) -> float:
    """Liquid-gas interface of the three-phase Stefan problem (Sec. 3.2): the
    frozen layer of thickness s was liquid of thickness s rho_s/rho_l, so the
    liquid column grows by s (1 - rho_s/rho_l); at full freezing H_f = H0 rho_l/rho_s."""
    s = neumann_front(ste, alpha_s, t)
    return H0 + (1.0 - ratio) * s


def enthalpy_1d(nx: int, nsteps: int, dt: float, latent: float, lam: float, rho: float, cp: float,
                T_wall: float, H0: np.ndarray) -> np.ndarray:
    """Textbook explicit enthalpy method in 1-D: compact second-order heat flux
    (lam/rho)(T_i - T_{i+1})/dx with dx = 1, a Dirichlet wall at x = 0 through a
    mirrored ghost (T_g = 2 T_wall - T_0), an adiabatic wall at x = nx, and the
    Shu-Osher SSP-RK3 scheme.  Melting point 0, single C_p, so
    T = min(H, 0)/cp + max(H - L, 0)/cp."""

    def temperature(H):
        return (np.minimum(H, 0.0) + np.maximum(H - latent, 0.0)) / cp

    def rate(H):
        T = temperature(H)
        Tg = 2.0 * T_wall - T[0]
        flux = np.empty(nx + 1)
        flux[0] = (lam / rho) * (Tg - T[0])
        flux[1:nx] = (lam / rho) * (T[:-1] - T[1:])
        flux[nx] = 0.0
        return -(flux[1:] - flux[:-1])

    H = H0.astype(np.float64).copy()
    for _ in range(nsteps):
        H1 = H + dt * rate(H)
        H2 = 0.75 * H + 0.25 * H1 + 0.25 * dt * rate(H1)
        H = H / 3.0 + 2.0 / 3.0 * H2 + 2.0 / 3.0 * dt * rate(H2)
    return H


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b.ravel())
    num = np.linalg.norm((a - b).ravel())
    return float(num / den) if den > 0 else float(num)
