"""The allocation-free residual entry point (eulbfs_residual_noalloc) against
eulbfs_residual: the same kernels with the scratch in the library's static
device array instead of a temporary allocation, so the outputs are equal bit for
bit.  Two calls in a row, the second on a smaller grid (the static array keeps
the first call's contents), in FP64 and FP32; a grid beyond the array's size is
rejected."""
import numpy as np
import pytest

from paper_2507_03366_amd import eulbfs as E, problems as PB

pytestmark = pytest.mark.gpu


def _pair(pr, st):
    s = E.Solver(pr, st, kernel=E.KERNEL_FUSED)
    try:
        ref = s.residual()
        got = E.eulbfs_residual_noalloc(s.h, pr.nx, pr.ny)
    finally:
        s.close()
    return ref, got


@pytest.mark.parametrize("precision", [E.FP64, E.FP32])
def test_noalloc_residual_equals_residual(precision):
    big = PB.static_droplet(n=160, R=40)
    small = PB.film_freezing(n=72)
    for pr, st in (big, small):
        pr = pr.replace(precision=precision)
        ref, got = _pair(pr, st)
        for a, b in zip(ref, got):
            assert a.shape == b.shape
            assert np.isfinite(a).all()
            assert np.array_equal(a, b)


def test_noalloc_rejects_a_grid_beyond_the_scratch():
    pr, st = PB.static_droplet(n=1024, R=256)
    s = E.Solver(pr, st, kernel=E.KERNEL_FUSED)
    try:
        with pytest.raises(E.EulbfsError) as ei:
            E.eulbfs_residual_noalloc(s.h, pr.nx, pr.ny)
        assert ei.value.code == E.EINVAL
    finally:
        s.close()
