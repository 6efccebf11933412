"""Randomised parity: seeded random problems (grid size, every wall rule per
side, periodic directions, lattice, mushy range, phase properties, surface
force model, the C-source reading, gravity, a random drop or layer with noisy
temperature) run on the GPU and in the oracle for 60 steps, equal to 1e-10
relative L2 per field.  The seeds cycle through every fused tile shape and the
split kernels.  Problems the parameter check rejects are redrawn.

A draw can leave a field so small that rounding alone moves it by more than
that bar (a fully periodic box whose pressure stays below 4e-7 in lattice units):
the oracle's own response to a one-ulp change of every input value measures
this, and such a field's bar is 100 times that response (the two sides round
differently at each of the 60 steps, not only at the first)."""
import copy

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


def _random_problem(rng):
    while True:
        nx, ny = int(rng.integers(20, 91)), int(rng.integers(20, 91))
        px, py = bool(rng.random() < 0.25), bool(rng.random() < 0.25)
        walls = {}
        for side in PB.SIDES:
            flow = int(rng.choice([PB.NOSLIP, PB.FREESLIP, PB.OUTLET]))
            heat = int(rng.choice([PB.ADIABATIC, PB.DIRICHLET]))
            theta = float(rng.uniform(45.0, 135.0))
            adv = rec = 0.0
            if rng.random() < 0.3:
                rec, adv = theta - float(rng.uniform(5, 30)), theta + float(rng.uniform(5, 30))
            walls[side] = PB.Wall(flow, heat, float(rng.uniform(-1.0, 0.5)), theta, adv, rec)
        rho_g = float(rng.uniform(0.02, 0.5))
        ratio = float(rng.uniform(0.85, 1.15))
        cp = (float(rng.uniform(0.5, 1.5)), 1.0, float(rng.uniform(0.5, 1.5)))
        lam_l = float(rng.uniform(0.05, 0.3))
        lam = (lam_l * float(rng.uniform(0.5, 3.0)), lam_l, lam_l * rho_g)
        mu_l = float(rng.uniform(0.02, 0.1))
        T_s = float(rng.uniform(-0.2, 0.0)) if rng.random() < 0.4 else 0.0
        T_l = float(rng.uniform(0.0, 0.2)) if T_s < 0 else 0.0
        pr = PB.Problem(
            nx=nx, ny=ny, lattice_hg=int(rng.choice([5, 9])), rho=(ratio, 1.0, rho_g), mu=(mu_l, mu_l, mu_l * rho_g),
            lam=lam, cp=cp, latent=float(rng.uniform(2.0, 20.0)), T_s=T_s, T_l=T_l,
            sigma=float(rng.uniform(0.0, 0.01)), gx=float(rng.uniform(-1e-5, 1e-5)), gy=float(rng.uniform(-1e-5, 0)),
            surf_model=int(rng.integers(0, 2)), c_source=int(rng.integers(0, 2)), periodic_x=px, periodic_y=py,
            walls=walls)
        if E.eulbfs_check_params(E.params_from_problem(pr)):
            continue
        if rng.random() < 0.5:
            sh = PB.Shape(profile=PB.PROFILE_DROPLET, x0=float(rng.uniform(0.3, 0.7) * nx),
                          y0=float(rng.uniform(0.0, 0.5) * ny), r0=float(rng.uniform(0.2, 0.4) * min(nx, ny)),
                          t_in=float(rng.uniform(-0.3, 0.3)), t_out=float(rng.uniform(-0.3, 0.3)),
                          t_amp=0.01, seed=int(rng.integers(0, 2 ** 31)), u_in=float(rng.uniform(-0.01, 0.01)),
                          v_in=float(rng.uniform(-0.01, 0.01)))
        else:
            sh = PB.Shape(profile=PB.PROFILE_LAYER, axis=int(rng.integers(0, 2)),
                          h0=float(rng.uniform(0.3, 0.7)) * (nx if rng.random() < 0.5 else ny),
                          t_in=float(rng.uniform(-0.3, 0.3)), t_out=float(rng.uniform(-0.3, 0.3)), t_amp=0.01,
                          seed=int(rng.integers(0, 2 ** 31)))
        return pr, sh.state(pr)


PATHS = [(E.KERNEL_FUSED, t) for t in ((32, 8), (64, 4), (16, 16), (64, 8), (32, 16), (32, 32))] + [
    (E.KERNEL_SPLIT, (0, 0))]


GROUPS = (("H", [0]), ("p", [1]), ("M", [2, 3]), ("C", [4]))


def _rel(a, b):
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / den) if den > 0 else float(np.abs(a).max())


def _ulp_response(oracle, pr, st, steps, Wref, seed):
    """relative change of each field group after `steps` when every input
    value is multiplied by 1 + 2.2e-16 * N(0, 1)"""
    st2 = copy.deepcopy(st)
    r = np.random.default_rng(seed)
    for name in ("T", "Fl", "C", "u", "v", "p"):
        a = getattr(st2, name)
        setattr(st2, name, a * (1 + 2.2e-16 * r.standard_normal(a.shape)))
    W2, _ = oracle.run(pr, st2, steps)
    return {name: _rel(W2[ks], Wref[ks]) for name, ks in GROUPS}


@pytest.mark.parametrize("seed", range(42))
def test_random_problem_matches_oracle(oracle, seed):
    rng = np.random.default_rng(1000 + seed)
    pr, st = _random_problem(rng)
    oracle.set_threads(16)
    Wref, _ = oracle.run(pr, st, 60)
    if not np.all(np.isfinite(Wref)):
        pytest.skip("the oracle itself went non-finite on this draw")
    kernel, tile = PATHS[seed % len(PATHS)]
    s = E.Solver(pr, st, kernel=kernel, tile=tile)
    try:
        s.step(60)
        w = s.conserved()
    finally:
        s.close()
    resp = _ulp_response(oracle, pr, st, 60, Wref, seed)
    for name, ks in GROUPS:
        err = _rel(w[ks], Wref[ks])
        assert err <= max(1e-10, 100 * resp[name]), (seed, kernel, tile, name, err, resp[name], pr)
