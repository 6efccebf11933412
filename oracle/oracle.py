"""ctypes wrapper of the FP64 CPU oracle (liboracle.so built from eulbfs_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The product path never imports it.
Arrays are float64; W is (5, ny, nx) = (H, p, rho c_s^2 u, rho c_s^2 v, C).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "eulbfs_oracle.c")


def build(force: bool = True) -> str:
    """Compile the oracle (gcc, FP64, no FMA contraction, OpenMP over rows)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O3", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
               "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _BC(ct.Structure):
    _fields_ = [("periodic", ct.c_int32), ("flow", ct.c_int32), ("heat", ct.c_int32),
                ("pad", ct.c_int32), ("T_w", ct.c_double), ("theta_deg", ct.c_double),
                ("theta_adv", ct.c_double), ("theta_rec", ct.c_double)]


class _Params(ct.Structure):
    _fields_ = [
        ("nx", ct.c_int32), ("ny", ct.c_int32), ("lattice_hg", ct.c_int32), ("surf_model", ct.c_int32),
        ("c_source", ct.c_int32), ("pad", ct.c_int32),
        ("dx", ct.c_double), ("delta_t", ct.c_double), ("dt", ct.c_double),
        ("rho", ct.c_double * 3), ("mu", ct.c_double * 3), ("lam", ct.c_double * 3), ("cp", ct.c_double * 3),
        ("latent", ct.c_double), ("T_s", ct.c_double), ("T_l", ct.c_double),
        ("sigma", ct.c_double), ("xi", ct.c_double), ("mobility", ct.c_double), ("Qg", ct.c_double),
        ("gx", ct.c_double), ("gy", ct.c_double),
        ("bc", _BC * 4),
        ("xw", ct.POINTER(ct.c_double)), ("yw", ct.POINTER(ct.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ct.CDLL(_LIB_PATH)
        dp = ct.POINTER(ct.c_double)
        pp = ct.POINTER(_Params)
        L.or_closure.argtypes = [pp, ct.c_double, ct.c_double, dp, dp]
        L.or_closure.restype = None
        L.or_equilibria.argtypes = [pp] + [ct.c_double] * 9 + [dp, dp, dp]
        L.or_equilibria.restype = None
        L.or_init.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp]
        L.or_ghosts.argtypes = [pp, dp, dp]
        L.or_residual.argtypes = [pp, dp, dp, dp, dp, dp]
        L.or_step.argtypes = [pp, dp, dp, ct.c_int64]
        L.or_primitives.argtypes = [pp, dp, dp]
        L.or_diagnostics.argtypes = [pp, dp, dp]
        L.or_set_threads.argtypes = [ct.c_int]
        L.or_set_threads.restype = None
        for name in ("or_init", "or_ghosts", "or_residual", "or_step", "or_primitives", "or_diagnostics",
                     "or_num_threads"):
            getattr(L, name).restype = ct.c_int
        _lib = L
    return _lib


def params(pr) -> _Params:
    """Map a problems.Problem onto the oracle's parameter struct."""
    P = _Params()
    P.nx, P.ny, P.lattice_hg, P.surf_model = pr.nx, pr.ny, pr.lattice_hg, pr.surf_model
    P.c_source = pr.c_source
    P.dx, P.delta_t, P.dt = pr.dx, pr.delta_t, pr.dt
    for name in ("rho", "mu", "lam", "cp"):
        getattr(P, name)[:] = list(getattr(pr, name))
    P.latent, P.T_s, P.T_l = pr.latent, pr.T_s, pr.T_l
    P.sigma, P.xi, P.mobility, P.Qg = pr.sigma, pr.xi, pr.mobility, pr.Qg
    P.gx, P.gy = pr.gx, pr.gy
    for k, side in enumerate(("x-", "x+", "y-", "y+")):
        w = pr.wall(side)
        if w is None:
            P.bc[k].periodic = 1
        else:
            P.bc[k].periodic = 0
            P.bc[k].flow, P.bc[k].heat = w.flow, w.heat
            P.bc[k].T_w, P.bc[k].theta_deg = w.T_w, w.theta_deg
            P.bc[k].theta_adv, P.bc[k].theta_rec = w.theta_adv, w.theta_rec
    # stretched mesh (R24): the arrays stay referenced by the struct
    P._widths = []
    for name, src, n in (("xw", pr.x_width, pr.nx), ("yw", pr.y_width, pr.ny)):
        if src is not None:
            a = np.ascontiguousarray(src, dtype=np.float64)
            if a.shape != (n,):
                raise ValueError(f"{name}: expected {n} widths, got shape {a.shape}")
            P._widths.append(a)
            setattr(P, name, a.ctypes.data_as(ct.POINTER(ct.c_double)))
    return P


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _check(rc):
    if rc != 0:
        raise ValueError(f"oracle rejected the parameters (rc={rc})")


def closure(pr, H: float, C: float):
    Fl, T = ct.c_double(), ct.c_double()
    lib().or_closure(ct.byref(params(pr)), H, C, ct.byref(Fl), ct.byref(T))
    return Fl.value, T.value


def equilibria(pr, H, T, cp, p, rho, C, muc, u, v):
    h = np.zeros(9)
    f = np.zeros(9)
    g = np.zeros(9)
    lib().or_equilibria(ct.byref(params(pr)), H, T, cp, p, rho, C, muc, u, v, _ptr(h), _ptr(f), _ptr(g))
    q = 5 if pr.lattice_hg == 5 else 9
    return h[:q], f, g[:q]


def init(pr, state) -> np.ndarray:
    T, Fl, C, u, v, p = state.planes()
    W = np.zeros((5, pr.ny, pr.nx))
    _check(lib().or_init(ct.byref(params(pr)), _ptr(T), _ptr(Fl), _ptr(C), _ptr(u), _ptr(v), _ptr(p), _ptr(W)))
    return W


def ghosts(pr, W: np.ndarray) -> np.ndarray:
    W = np.ascontiguousarray(W, dtype=np.float64)
    Wg = np.zeros((5, pr.ny + 6, pr.nx + 6))
    _check(lib().or_ghosts(ct.byref(params(pr)), _ptr(W), _ptr(Wg)))
    return Wg


def residual(pr, W: np.ndarray, Fsdot=None):
    """R(W) on the interior, with the x-face and y-face fluxes."""
    W = np.ascontiguousarray(W, dtype=np.float64)
    fs = np.zeros((pr.ny, pr.nx)) if Fsdot is None else np.ascontiguousarray(Fsdot, dtype=np.float64)
    R = np.zeros((5, pr.ny, pr.nx))
    Fx = np.zeros((5, pr.ny, pr.nx + 1))
    Fy = np.zeros((5, pr.ny + 1, pr.nx))
    _check(lib().or_residual(ct.byref(params(pr)), _ptr(W), _ptr(fs), _ptr(R), _ptr(Fx), _ptr(Fy)))
    return R, Fx, Fy


def step(pr, W: np.ndarray, Fsdot: np.ndarray, nsteps: int):
    """Advance (W, dF_s/dt) by nsteps SSP-RK3 steps; returns new arrays."""
    W = np.array(W, dtype=np.float64, order="C", copy=True)
    fs = np.array(Fsdot, dtype=np.float64, order="C", copy=True)
    _check(lib().or_step(ct.byref(params(pr)), _ptr(W), _ptr(fs), int(nsteps)))
    return W, fs


def primitives(pr, W: np.ndarray):
    """(T, F_l, F_s, rho, u, v, mu_c), each (ny, nx)."""
    W = np.ascontiguousarray(W, dtype=np.float64)
    out = np.zeros((7, pr.ny, pr.nx))
    _check(lib().or_primitives(ct.byref(params(pr)), _ptr(W), _ptr(out)))
    return out


def diagnostics(pr, W: np.ndarray):
    """[sum rho dV, sum C dV, sum H dV, sum F_s dV, max |u|]."""
    W = np.ascontiguousarray(W, dtype=np.float64)
    out = np.zeros(5)
    _check(lib().or_diagnostics(ct.byref(params(pr)), _ptr(W), _ptr(out)))
    return out


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def run(pr, state, nsteps: int):
    """Initial state -> (W, dF_s/dt) after nsteps."""
    W = init(pr, state)
    return step(pr, W, np.zeros((pr.ny, pr.nx)), nsteps)
