"""Tile shapes and the tile autotuner: every tile shape of the fused stage
kernel, and the shape EULBFS_KERNEL_AUTO picks at create, give the same bits
(the tile only changes which workgroup computes a cell), on ragged and
periodic grids, both lattices and both precisions; the timed trial steps
leave no trace in the state."""
import numpy as np
import pytest

from paper_2507_03366_amd import eulbfs as E
from paper_2507_03366_amd import problems as PB

pytestmark = pytest.mark.gpu

TILES = ((32, 8), (64, 4), (16, 16), (64, 8), (32, 16), (32, 32))


def _ragged(lattice_hg=9, periodic_x=False):
    # 97 x 61: partial tiles in both directions for every tile shape
    pr, _ = PB.static_droplet(n=64, R=16, lattice_hg=lattice_hg)
    pr = pr.replace(nx=97, ny=61, sigma=0.015625, periodic_x=periodic_x)
    X, Y = PB.cell_centres(pr)
    st = PB.uniform_state(pr)
    st.C = PB.droplet_profile(X, Y, 48.5, 0.0, 16.0, 4.0)
    return pr, st


CASES = {
    "ragged_d2q9": lambda: _ragged(),
    "ragged_d2q5_periodic_x": lambda: _ragged(lattice_hg=5, periodic_x=True),
    "stefan3_periodic_y": PB.three_phase_stefan,
    "impact48": lambda: PB.impact_droplet(n=48, we=20.0, re=200.0),
}


def _run(pr, st, precision, nsteps, kernel=E.KERNEL_FUSED, tile=(0, 0)):
    s = E.Solver(pr, st, precision=precision, kernel=kernel, tile=tile)
    try:
        s.step(nsteps)
        return s.conserved(), s.diagnostics(), s.schedule()
    finally:
        s.close()


@pytest.mark.parametrize("precision", [E.FP64, E.FP32])
@pytest.mark.parametrize("name", sorted(CASES))
def test_every_tile_shape_and_auto_give_the_same_bits(name, precision):
    pr, st = CASES[name]()
    ref, _, sched = _run(pr, st, precision, 30, tile=(32, 8))
    assert sched == (E.KERNEL_FUSED, 32, 8)
    for tile in TILES[1:]:
        w, _, sched = _run(pr, st, precision, 30, tile=tile)
        assert sched == (E.KERNEL_FUSED,) + tile
        assert np.array_equal(w, ref), (name, tile)
    w, d, sched = _run(pr, st, precision, 30, kernel=E.KERNEL_AUTO)
    assert sched[0] == E.KERNEL_FUSED and sched[1:] in TILES
    assert d["steps"] == 30  # the trial steps were undone by re-initialising
    assert np.array_equal(w, ref), (name, "auto", sched)


def test_auto_choice_is_cached_per_grid():
    import time

    pr, st = PB.static_droplet(n=256, R=64)
    t0 = time.perf_counter()
    a = E.Solver(pr, st, kernel=E.KERNEL_AUTO)
    t1 = time.perf_counter()
    b = E.Solver(pr, st, kernel=E.KERNEL_AUTO)
    t2 = time.perf_counter()
    try:
        assert a.schedule() == b.schedule()
        print("create with tuning %.1f ms, cached %.1f ms" % ((t1 - t0) * 1e3, (t2 - t1) * 1e3))
    finally:
        a.close()
        b.close()
