"""Continuous-batching server: requests that arrive while others run are
admitted as slots and arena bytes free up, and every request finishes with
its full step budget and a finite state."""
import numpy as np
import pytest

from paper_2507_03366_amd import eulbfs as E
from paper_2507_03366_amd import serve as S

pytestmark = pytest.mark.gpu


def test_serving_burst_and_poisson():
    reqs = S.draw_requests(12, seed=3, nsteps=150, sizes=(64, 128))
    # a small arena and few slots force requests to wait for earlier ones
    st = S.serve(reqs, hbm_budget=48 << 20, max_slots=4, tick_steps=40)
    assert st["failed"] == []
    assert st["solves"] == 12 and st["p99_s"] >= st["p50_s"] > 0
    reqs2 = S.draw_requests(12, seed=3, nsteps=150, sizes=(64, 128))
    for r, a in zip(reqs2, S.poisson_arrivals(12, rate=40.0, seed=4)):
        r.arrival = float(a)
    st2 = S.serve(reqs2, hbm_budget=48 << 20, max_slots=4, tick_steps=40)
    assert st2["failed"] == []


def test_served_result_equals_the_request_alone():
    """A request finished in a busy mix holds exactly the state it reaches
    when it is the only request of a batch."""
    import torch

    reqs = S.draw_requests(6, seed=5, nsteps=120, sizes=(64, 128))
    target = reqs[2]
    pr, st = S.build(target, E.FP32)
    alone = E.Batch(64 << 20, 2, precision=E.FP32, stream=torch.cuda.Stream())
    s = alone.admit(pr, st, target.nsteps)
    while alone.diagnostics(s)["steps"] < target.nsteps:
        alone.tick(50)
    w_alone = alone.conserved(s)
    alone.close()
    mix = E.Batch(256 << 20, 8, precision=E.FP32, stream=torch.cuda.Stream())
    slots = []
    for r in reqs:
        p2, s2 = S.build(r, E.FP32)
        slots.append(mix.admit(p2, s2, r.nsteps if r is not target else target.nsteps))
    while mix.diagnostics(slots[2])["steps"] < target.nsteps:
        mix.tick(30)
    w_mix = mix.conserved(slots[2])
    mix.close()
    assert np.array_equal(w_alone, w_mix)
