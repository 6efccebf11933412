"""Batched solves through the C ABI: many uneven grids advanced by one
persistent launch per RK stage.  Each request must match the FP64 oracle,
and must be bitwise the same alone in a batch and in a mix (the per-cell
arithmetic does not depend on the other requests)."""
import numpy as np
import pytest

from paper_2507_03366_amd import eulbfs as E
from paper_2507_03366_amd import problems as PB

pytestmark = pytest.mark.gpu

GROUPS = (("H", [0]), ("p", [1]), ("M", [2, 3]), ("C", [4]))


def rel_l2(a, b):
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / den) if den > 0 else float(np.linalg.norm(a.ravel()))


def errors(w, ref):
    return {k: rel_l2(w[ks], ref[ks]) for k, ks in GROUPS}


def _requests():
    reqs = []
    pr, st = PB.static_droplet(n=64, R=16)
    reqs.append((pr.replace(sigma=0.015625), st))
    pr, st = PB.static_droplet(n=64, R=16, lattice_hg=5)
    pr = pr.replace(nx=90, ny=70, sigma=0.015625)
    X, Y = PB.cell_centres(pr)
    st = PB.uniform_state(pr)
    st.C = PB.droplet_profile(X, Y, 45.0, 0.0, 18.0, 4.0)
    reqs.append((pr, st))
    reqs.append(PB.three_phase_stefan())
    reqs.append(PB.conductive_freezing())
    reqs.append(PB.impact_droplet(n=48, we=20.0, re=200.0))
    return reqs


def _run_batch(reqs, nsteps, precision=E.FP64, tick=10, budget=1 << 28, tile=E.BATCH_TILE_AUTO, schedule=None):
    import torch

    b = E.Batch(budget, 16, precision=precision, stream=torch.cuda.Stream())
    try:
        b.set_tile(tile)
        slots = [b.admit(pr, st, n) for (pr, st), n in zip(reqs, nsteps)]
        assert all(s is not None for s in slots)
        while True:
            pending = [s for s, n in zip(slots, nsteps) if b.diagnostics(s)["steps"] < n]
            if not pending:
                break
            b.tick(tick)
        torch.cuda.synchronize()
        done = set(b.poll())
        assert done == set(slots)
        out = [b.conserved(s) for s in slots]
        diags = [b.diagnostics(s) for s in slots]
        if schedule is not None:
            schedule.append(b.schedule())
        for s in slots:
            b.release(s)
    finally:
        b.close()
    return out, diags


def test_batch_matches_oracle_and_is_independent_of_the_mix(oracle):
    reqs = _requests()
    nsteps = [100, 80, 100, 60, 100]
    mix, diags = _run_batch(reqs, nsteps)
    oracle.set_threads(16)
    for (pr, st), n, w, d in zip(reqs, nsteps, mix, diags):
        assert d["steps"] == n
        Wref, fsref = oracle.run(pr, st, n)
        errs = errors(w[:5], Wref)
        assert max(errs.values()) < 1e-11, (pr.nx, pr.ny, errs)
    # each request alone in a batch: bitwise equal to its result in the mix
    for k in (0, 1, 4):
        alone, _ = _run_batch([reqs[k]], [nsteps[k]])
        assert np.array_equal(alone[0], mix[k]), k


def test_batch_full_size_requests_match_oracle(oracle):
    """Serving-mix grids at their full sizes: a 512 x 512 impact and a 256 x 256
    static droplet in one FP64 batch, 10 steps against the oracle."""
    reqs = [PB.impact_droplet(n=512, we=50.0, re=1000.0, ste=0.5, supercool=0.5, theta_deg=70.0),
            PB.static_droplet(n=256, R=64, theta_deg=110.0, ste=0.3)]
    reqs[1] = (reqs[1][0].replace(sigma=PB.static_droplet()[0].sigma), reqs[1][1])
    out, diags = _run_batch(reqs, [10, 10], tick=5, budget=1 << 30)
    oracle.set_threads(16)
    for (pr, st), w, d in zip(reqs, out, diags):
        assert d["steps"] == 10
        Wref, _ = oracle.run(pr, st, 10)
        errs = errors(w[:5], Wref)
        assert max(errs.values()) < 1e-12, (pr.nx, errs)


def test_empty_batch_tick_and_poll():
    import torch

    b = E.Batch(1 << 26, 4, precision=E.FP32, stream=torch.cuda.Stream())
    try:
        b.tick(10)  # nothing resident: no launch, no error
        assert b.poll() == []
    finally:
        b.close()


def test_batch_agrees_with_single_solver():
    pr, st = PB.static_droplet(n=64, R=16)
    pr = pr.replace(sigma=0.015625)
    w_b, _ = _run_batch([(pr, st)], [50])
    s = E.Solver(pr, st, tile=(32, 8))
    s.step(50)
    w_s = s.conserved()
    s.close()
    assert max(errors(w_b[0][:5], w_s[:5]).values()) < 1e-13


def test_batch_fp32_against_oracle(oracle):
    reqs = _requests()[:3]
    nsteps = [200, 200, 200]
    out, _ = _run_batch(reqs, nsteps, precision=E.FP32)
    oracle.set_threads(16)
    for (pr, st), n, w in zip(reqs, nsteps, out):
        Wref, _ = oracle.run(pr, st, n)
        errs = errors(w[:5], Wref)
        assert max(errs.values()) < 1e-4, errs


def test_batch_admission_by_footprint():
    import torch

    pr, st = PB.static_droplet(n=256, R=64)
    need = E.eulbfs_batch_request_bytes(E.params_from_problem(pr, precision=E.FP64))
    b = E.Batch(int(need * 1.5) + (1 << 20), 8, precision=E.FP64, stream=torch.cuda.Stream())
    try:
        s0 = b.admit(pr, st, 10)
        assert s0 is not None
        assert b.admit(pr, st, 10) is None  # second copy does not fit
        small, sst = PB.static_droplet(n=64, R=16, sigma=0.015625)
        s1 = b.admit(small, sst, 10)        # a small one still fits beside it
        assert s1 is not None
        b.release(s0)
        s2 = b.admit(pr, st, 10)            # the freed range is reused
        assert s2 is not None
        # a request of another precision is refused
        with pytest.raises(E.EulbfsError):
            E.eulbfs_batch_admit(b.b, E.params_from_problem(small, precision=E.FP32),
                                 np.concatenate([a.ravel() for a in sst.planes()]), 10)
    finally:
        b.close()


def test_graph_replay_matches_eager_launches():
    """Steps replayed from a captured graph (created stream) equal eager
    launches on the default stream, across several calls with host work and
    queries between the replays."""
    import torch

    pr, st = PB.film_freezing(n=64)
    a = E.Solver(pr, st, stream=torch.cuda.Stream())
    b = E.Solver(pr, st)  # legacy default stream: eager launches
    try:
        for n in (40, 16, 33, 64):
            a.step(n)
            b.step(n)
            wa, wb = a.conserved(), b.conserved()
            assert np.array_equal(wa, wb), n
    finally:
        a.close()
        b.close()


def test_batch_step_graphs_match_eager_ticks():
    """Ticks replayed from captured step graphs (a created stream) equal eager
    ticks (the legacy default stream, where nothing is captured) bit for bit
    while the resident set changes: a request finishes and another is admitted
    between ticks, so the graphs are captured again; every replay is checked
    after the host has synchronised and queried."""
    import torch

    reqs = _requests()

    def drive(stream):
        b = E.Batch(1 << 28, 8, precision=E.FP64, stream=stream)
        seen = []
        try:
            a = b.admit(*reqs[0], 80)
            c = b.admit(*reqs[3], 30)
            for k in range(8):
                if k == 2:
                    d = b.admit(*reqs[1], 40)
                b.tick(10)
                torch.cuda.synchronize()
                seen.append(b.conserved(a))
                if k >= 2:
                    seen.append(b.conserved(d))
            seen.append(b.conserved(c))
        finally:
            b.close()
        return seen

    captured = drive(torch.cuda.Stream())
    eager = drive(None)
    assert len(captured) == len(eager)
    for x, y in zip(captured, eager):
        assert np.array_equal(x, y)


def _graded_request():
    wx = PB.graded_widths(60, 0.6, 1.04, 1.5, both_ends=True)
    wy = PB.graded_widths(45, 0.6, 1.05, 1.5)
    pr = PB.Problem(nx=60, ny=45, x_width=wx, y_width=wy, rho=(0.917, 1.0, 0.01), mu=(0.05, 0.05, 0.0005),
                    lam=(0.4, 0.4, 0.004), latent=10.0, sigma=0.005, gy=-1e-5, delta_t=0.3, dt=0.3,
                    walls={"y-": PB.Wall(PB.NOSLIP, PB.DIRICHLET, -1.0, 75.0), "y+": PB.Wall(PB.FREESLIP),
                           "x-": PB.Wall(), "x+": PB.Wall()})
    X, Y = PB.cell_centres(pr)
    st = PB.uniform_state(pr, T0=0.1)
    st.C = PB.droplet_profile(X, Y, 0.5 * wx.sum(), 0.0, 15.0, pr.xi)
    return pr, st


@pytest.mark.parametrize("precision", [E.FP64, E.FP32])
def test_batch_tile_shapes_give_the_same_bits(precision):
    """The uneven mix plus a stretched request with the batch tile pinned to
    32x16, pinned to 64x8 and chosen on the fly: every request bitwise the same.
    After ten ticks the automatic choice has timed both shapes on back-to-back
    ticks of the same work."""
    reqs = _requests() + [_graded_request()]
    nsteps = [100, 80, 100, 60, 100, 90]
    a, _ = _run_batch(reqs, nsteps, precision=precision, tile=E.BATCH_TILE_32x16)
    b, _ = _run_batch(reqs, nsteps, precision=precision, tile=E.BATCH_TILE_64x8)
    sched = []
    c, _ = _run_batch(reqs, nsteps, precision=precision, tile=E.BATCH_TILE_AUTO, schedule=sched)
    for k in range(len(reqs)):
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c[k]), k
    sc = sched[0]
    assert min(sc["ticks_timed"]) >= 1 and min(sc["ns_per_cell_step"]) > 0
    assert sc["pairs"] >= 1 and sc["time_ratio"] > 0
    assert sc["next_tile"] in (E.BATCH_TILE_32x16, E.BATCH_TILE_64x8)


def test_batch_tile_choice_rejects_unknown_values():
    import torch

    b = E.Batch(1 << 26, 2, precision=E.FP32, stream=torch.cuda.Stream())
    try:
        for bad in (-1, 3):
            with pytest.raises(E.EulbfsError) as ei:
                b.set_tile(bad)
            assert ei.value.code == E.EINVAL
        b.set_tile(E.BATCH_TILE_64x8)
        assert b.schedule()["next_tile"] == E.BATCH_TILE_64x8
        b.set_tile(E.BATCH_TILE_AUTO)
        sc = b.schedule()  # nothing timed yet: tick 0 runs 32x16
        assert sc["next_tile"] == E.BATCH_TILE_32x16 and sc["pairs"] == 0 and sc["ticks_timed"] == [0, 0]
    finally:
        b.close()


def test_unstable_request_is_reported_and_isolated():
    """A request whose state holds a non-finite value runs in a batch beside a
    healthy one: its diagnostics report EULBFS_EUNSTABLE once it finishes, and
    the healthy request ends bitwise where it ends alone."""
    import torch

    pr, st = PB.static_droplet(n=64, R=16, sigma=0.015625)
    bad = PB.InitialState(T=st.T.copy(), Fl=st.Fl.copy(), C=st.C.copy(), u=st.u.copy(), v=st.v.copy(),
                          p=st.p.copy())
    bad.C[20, 30] = np.nan
    b = E.Batch(1 << 27, 4, precision=E.FP64, stream=torch.cuda.Stream())
    try:
        s_good = b.admit(pr, st, 60)
        s_bad = b.admit(pr, bad, 60)
        while len(b.poll()) < 2:
            b.tick(20)
        with pytest.raises(E.EulbfsError) as ei:
            b.diagnostics(s_bad)
        assert ei.value.code == E.EUNSTABLE and "non-finite" in str(ei.value)
        d = b.diagnostics(s_good)
        assert d["nonfinite"] == 0 and d["steps"] == 60
        w_good = b.conserved(s_good)
    finally:
        b.close()
    alone, _ = _run_batch([(pr, st)], [60], tick=20)
    assert np.array_equal(alone[0], w_good)


def test_batch_tile_choice_without_paired_ticks():
    """Ticks that never repeat their work (the step count changes every tick)
    give no paired sample: the choice alternates for 32 timed ticks of each
    shape, then follows the summed time per cell-step, with every eighth tick
    on the other shape."""
    import torch

    pr, st = PB.static_droplet(n=128, R=32, sigma=0.015625)
    b = E.Batch(1 << 28, 4, precision=E.FP32, stream=torch.cuda.Stream())
    try:
        b.admit(pr, st, 100000)
        for k in range(72):
            b.tick(3 + k % 5 + (k // 5) % 2)  # consecutive ticks always differ
        torch.cuda.synchronize()
        sc = b.schedule()
        assert sc["pairs"] == 0 and min(sc["ticks_timed"]) >= 32
        ns = sc["ns_per_cell_step"]
        best = E.BATCH_TILE_64x8 if ns[1] < ns[0] else E.BATCH_TILE_32x16
        other = E.BATCH_TILE_32x16 + E.BATCH_TILE_64x8 - best
        assert sc["next_tile"] == (other if 72 % 8 == 7 else best)
    finally:
        b.close()
