"""Parameter validation of the C ABI under random inputs (CPU, no device):
every parameter set is either accepted with a positive workspace size or
rejected with a message and a zero size, and a rejected set makes create
fail with EINVAL before any device call."""
import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from paper_2507_03366_amd import eulbfs as E
from paper_2507_03366_amd import problems as PB

BASE, _ = PB.static_droplet(n=64, R=16, sigma=0.015625)

finite = st.floats(min_value=-10.0, max_value=10.0, allow_nan=False)
anyfloat = st.one_of(finite, st.sampled_from([0.0, -1.0, 1e-300, 1e300, math.inf, -math.inf, math.nan]))


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(nx=st.integers(-2, 600), ny=st.integers(-2, 600), dx=anyfloat, delta_t=anyfloat, dt=anyfloat,
       rho=st.tuples(anyfloat, anyfloat, anyfloat), mu=st.tuples(anyfloat, anyfloat, anyfloat),
       sigma=anyfloat, xi=anyfloat, latent=anyfloat, lattice=st.sampled_from([5, 9, 7, 0]),
       precision=st.sampled_from([0, 1, 2, -1]), theta=anyfloat)
def test_random_parameters_are_accepted_or_rejected_cleanly(nx, ny, dx, delta_t, dt, rho, mu, sigma, xi, latent,
                                                            lattice, precision, theta):
    walls = dict(BASE.walls)
    w = walls["y-"]
    walls["y-"] = PB.Wall(w.flow, w.heat, w.T_w, theta)
    pr = BASE.replace(nx=nx, ny=ny, dx=dx, delta_t=delta_t, dt=dt, rho=rho, mu=mu, sigma=sigma, xi=xi,
                      latent=latent, lattice_hg=lattice, walls=walls)
    try:
        P = E.params_from_problem(pr, precision=precision)
    except (ValueError, OverflowError, TypeError):
        return  # not expressible in the C struct (the binding refuses it)
    msg = E.eulbfs_check_params(P)
    nbytes = E.eulbfs_workspace_bytes(P)
    if msg:
        assert nbytes == 0
        with pytest.raises(E.EulbfsError) as ei:
            E.eulbfs_create(P, np.zeros(6 * max(nx, 1) * max(ny, 1)))
        assert ei.value.code == E.EINVAL
    else:
        assert nx >= 4 and ny >= 4 and 0 < delta_t <= 0.5 * dx and dt > 0 and precision in (0, 1)
        assert all(math.isfinite(v) and v > 0 for v in rho) and xi >= 2 * dx
        assert nbytes >= 11 * nx * ny * (8 if precision == 0 else 4)


@settings(max_examples=200, deadline=None)
@given(nx=st.integers(4, 300), ny=st.integers(4, 300), scale=st.floats(0.5, 2.0), ratio=st.floats(0.8, 1.2),
       rho_g=st.floats(1e-3, 1.0), lattice=st.sampled_from([5, 9]), precision=st.sampled_from([0, 1]),
       theta=st.floats(10.0, 170.0))
def test_nearby_valid_parameters_size_their_workspace(nx, ny, scale, ratio, rho_g, lattice, precision, theta):
    """Parameter sets near a valid one: accepted unless an explicit step limit
    or range is broken, and the workspace grows with the grid and the field
    size."""
    walls = dict(BASE.walls)
    w = walls["y-"]
    walls["y-"] = PB.Wall(w.flow, w.heat, w.T_w, theta)
    pr = BASE.replace(nx=nx, ny=ny, rho=(ratio, 1.0, rho_g), mu=tuple(m * scale for m in BASE.mu),
                      lattice_hg=lattice, walls=walls)
    P = E.params_from_problem(pr, precision=precision)
    msg = E.eulbfs_check_params(P)
    if msg:
        assert "limit" in msg or "step" in msg, msg  # only the stability bounds can reject these
        return
    n = E.eulbfs_workspace_bytes(P)
    assert n >= 11 * nx * ny * (8 if precision == 0 else 4)
    # rows are padded to 256 bytes: a grid wider by 128 cells needs more
    P2 = E.params_from_problem(pr.replace(nx=nx + 128), precision=precision)
    if not E.eulbfs_check_params(P2):
        assert E.eulbfs_workspace_bytes(P2) > n
