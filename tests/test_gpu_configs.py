"""The benchmark configurations at full length on the GPU, against what the paper
and the mathematics fix, and FP32 mode against FP64 on each.

- Conductive freezing (Sec. 3.1, one-phase, 128 x 4): 20 000 steps on the D2Q9
  and the D2Q5 enthalpy lattice; at rest the two carry the same heat flux, so
  the runs agree to rounding and both fronts are the Neumann one (27.83 cells).
- Three-phase Stefan problem (Sec. 3.2, 256 x 8, rho_s/rho_l = 0.9): the full
  50 000 steps; the liquid-gas interface against H_0 + (1 - r) s with s the
  Neumann front (132.64 cells), the front against 2 k sqrt(alpha_s t).
- Film (Sec. 3.3, 256 x 256) to full freezing in FP32 mode and in FP64: time to
  solution and the FP64 volume balance of Eqs. (26) and (40).
- Static droplet (Sec. 3.4, 512 x 512): ice-tip height and solid volume every
  1000 steps, FP32 batched (one request in a batch, as served) against FP64
  on its own solver.
"""
import time

import numpy as np
import pytest

import analytic as A
from paper_2507_03366_amd import eulbfs as E
from paper_2507_03366_amd import problems as PB

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    E.lib()
    yield


def _rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _stream():
    import torch

    return torch.cuda.Stream()  # a created stream: the solver replays captured steps


def _timed_run(s, n):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.run(n)
    s.diagnostics()  # waits for the handle's stream
    return time.perf_counter() - t0


def test_conductive_freezing_d2q5_and_d2q9_full_length():
    """20 000 steps of Sec. 3.1 on each enthalpy lattice: the states agree to
    1e-12 relative L2 (only the rounding order of the face sums differs) and
    the front dx sum F_s / N_y is within 0.5 cell of 2 k sqrt(alpha t) = 27.83."""
    pr, st = PB.conductive_freezing()
    out = {}
    for q in (9, 5):
        s = E.Solver(pr.replace(lattice_hg=q), st, kernel=E.KERNEL_AUTO, stream=_stream())
        try:
            wall = _timed_run(s, 20000)
            out[q] = (s.conserved(), s.diagnostics())
        finally:
            s.close()
        print(f"D2Q{q}: front {out[q][1]['solid'] / pr.ny:.4f}, {pr.cells * 20000 / wall / 1e6:.1f} MLUPS "
              f"({wall / 20000 * 1e6:.2f} us/step)")
    front = A.neumann_front(0.1, 0.4, 20000 * pr.dt)
    assert front == pytest.approx(27.83, abs=0.01)
    assert _rel_l2(out[5][0][0], out[9][0][0]) < 1e-12
    for q in (9, 5):
        assert abs(out[q][1]["solid"] / (pr.ny * pr.dx) - front) < 0.5


@pytest.mark.parametrize("precision", [E.FP64, E.FP32])
def test_three_phase_stefan_full_length(precision):
    """50 000 steps (t = 25 000): the liquid-gas interface X_lg = dx sum C / N_y
    within 0.5 cell of 128 + 0.1 s(t) = 132.64 and the front X = dx sum F_s / N_y
    within 0.5 cell of the Neumann s(t) = 2 k sqrt(alpha_s t) = 46.4 (k(0.1) =
    0.2200163, alpha_s = 0.4 / 0.9), in FP64 and in FP32 mode."""
    pr, st = PB.three_phase_stefan()
    s = E.Solver(pr, st, precision=precision, kernel=E.KERNEL_AUTO, stream=_stream())
    try:
        wall = _timed_run(s, 50000)
        d = s.diagnostics()
    finally:
        s.close()
    t = 50000 * pr.dt
    alpha_s = pr.lam[0] / (pr.rho[0] * pr.cp[0])
    front = A.neumann_front(1.0 / pr.latent, alpha_s, t)
    x_lg = A.stefan_three_phase_interface(128.0, pr.rho[0], 1.0 / pr.latent, alpha_s, t)
    X_lg = d["volume_C"] / (pr.ny * pr.dx)
    X_f = d["solid"] / (pr.ny * pr.dx)
    print(f"precision {precision}: X_lg = {X_lg:.4f} (analytic {x_lg:.4f}), front {X_f:.4f} "
          f"(Neumann {front:.4f}), {pr.cells * 50000 / wall / 1e6:.1f} MLUPS ({wall / 50000 * 1e6:.2f} us/step)")
    assert x_lg == pytest.approx(132.64, abs=0.01)
    assert abs(X_lg - x_lg) < 0.5
    assert abs(X_f - front) < 0.5


def _film_to_full_freezing(precision, chunk=20000, limit=2_000_000):
    import torch

    pr, st = PB.film_freezing()
    s = E.Solver(pr, st, precision=precision, kernel=E.KERNEL_AUTO, stream=torch.cuda.Stream())
    try:
        d0 = s.diagnostics()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prev, steps = -1.0, 0
        while steps < limit:
            s.run(chunk)
            steps += chunk
            d = s.diagnostics()
            # frozen: the condensed phase is solid but for the gas side of the
            # interface, which freezes only as fast as the gas above it cools
            if d["solid"] > 0.999 * d["volume_C"] or (d["solid"] > 0.9 * d["volume_C"] and
                                                      d["solid"] - prev < 1e-6 * d0["volume_C"]):
                break
            prev = d["solid"]
        wall = time.perf_counter() - t0
        w = s.conserved()
    finally:
        s.close()
    return pr, d0, d, steps, wall, w


def test_film_to_full_freezing_fp32_and_fp64():
    """The 256 x 256 film until the condensed phase has frozen, in FP32 mode and
    in FP64.  The FP64 integrals keep the volume balance of Eqs. (26) and (40):
    the condensed volume grows by (1 - r) times the solid formed up to the step
    before the last (the source takes the lagged rate dF_s/dt), to rounding in
    FP64 (1e-10 of the volume); in FP32 mode, where that rate is stored and the
    C residual summed in FP32, to the FP32 rounding of all the solid formed,
    2^-24 (1 - r) times it, relative to the volume.
    The final volume is rho_l/rho_s times the initial one within 0.05 % once
    the gas side of the interface not yet frozen is allowed for; FP32 and FP64
    stop within one check interval of each other with the same final volume
    to 1e-4."""
    res = {}
    for prec in (E.FP32, E.FP64):
        pr, d0, d, steps, wall, w = _film_to_full_freezing(prec)
        r = pr.rho[0] / pr.rho[1]
        unfrozen = 1.0 - d["solid"] / d["volume_C"]
        S0 = d0["volume_C"]
        formed = d["solid"] - d0["solid"]
        last = pr.dt * float(w[5].sum()) * pr.dx * pr.dx  # solid formed in the last step
        drift = (d["volume_C"] - S0 - (1.0 - r) * (formed - last)) / S0
        S_n = d["volume_C"] / S0
        res[prec] = (steps, S_n, d)
        print(f"film precision {prec}: frozen after {steps} steps, {wall:.1f} s "
              f"({pr.cells * steps / wall / 1e6:.0f} MLUPS, {wall / steps * 1e6:.1f} us/step); S_n/S_0 = {S_n:.6f} "
              f"against rho_l/rho_s {1 / r:.6f}; volume-balance drift {drift:.2e} (last-step term "
              f"{(1.0 - r) * last / S0:.2e}); unfrozen {unfrozen:.4f}")
        assert steps < 2_000_000 and d["nonfinite"] == 0
        bar = 1e-10 + (2.0 ** -24 * (1.0 - r) * formed / S0 if prec == E.FP32 else 0.0)
        assert abs(drift) < bar
        assert abs(S_n * r - 1.0) < 5e-4 + (1.0 - r) * unfrozen
    assert abs(res[E.FP32][0] - res[E.FP64][0]) <= 20000
    assert res[E.FP32][1] == pytest.approx(res[E.FP64][1], rel=1e-4)


def test_droplet_fp32_batched_against_fp64():
    """The 512 x 512 droplet for 40 000 steps: ice-tip height (dy sum F_s up the
    middle column) and solid volume every 1000 steps, FP32 mode in a batch
    (as served) against FP64 on its own autotuned solver.  The tip agrees within
    0.5 cell (the serving bar) and the solid volume within 1e-4 relative at every
    sample; every conserved field within 1e-4 relative L2 at the end (the
    serving bar, here over 40 000 steps)."""
    import torch

    pr, st = PB.static_droplet()
    n, every = 40000, 1000
    s64 = E.Solver(pr, st, kernel=E.KERNEL_AUTO, stream=torch.cuda.Stream())
    b = E.Batch(1 << 30, 4, precision=E.FP32, stream=torch.cuda.Stream())
    hist = []
    try:
        slot = b.admit(pr, st, n)
        assert slot is not None
        for k in range(n // every):
            s64.run(every)
            b.tick(every)
            d64 = s64.diagnostics()
            d32 = b.diagnostics(slot)
            assert d32["steps"] == d64["steps"] == every * (k + 1)
            hist.append((d64["tip"], d32["tip"], d64["solid"], d32["solid"]))
        w64, w32 = s64.conserved(), b.conserved(slot)
    finally:
        s64.close()
        b.close()
    worst_tip = max(abs(h[1] - h[0]) for h in hist)
    worst_solid = max(abs(h[3] - h[2]) / h[2] for h in hist)
    for k in range(0, len(hist), 5):
        t64, t32, f64, f32 = hist[k]
        print(f"step {every * (k + 1)}: tip {t64:.4f} / {t32:.4f}, solid {f64:.3f} / {f32:.3f}")
    errs = {name: _rel_l2(w32[ks], w64[ks]) for name, ks in (("H", [0]), ("p", [1]), ("M", [2, 3]), ("C", [4]))}
    print(f"p of the FP64 run: rms {np.sqrt(np.mean(w64[1] ** 2)):.3e}, max |p| {np.abs(w64[1]).max():.3e}")
    print(f"worst tip difference {worst_tip:.2e} cells, worst solid {worst_solid:.2e}, final rel L2 {errs}")
    assert hist[-1][2] > hist[0][2] > 0  # the drop freezes from the wall up
    assert worst_tip < 0.5
    assert worst_solid <= 1e-4
    for name, e in errs.items():
        assert e <= 1e-4, name
