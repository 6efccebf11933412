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
