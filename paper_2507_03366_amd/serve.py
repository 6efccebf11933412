"""Continuous-batching server for EULBFS solve requests.

Requests arrive over time (Poisson arrivals), each a freezing droplet of its
own grid size and parameters (Stefan number, supercooling, contact angle; half
of them droplets impacting the cold wall at a drawn Weber and Reynolds
number).  The server keeps every admitted request resident in one device
arena (eulbfs_batch_*), admits waiting requests first-come first-served as
slots and arena bytes free up, advances all resident requests together by
one launch per RK stage per tick, and retires each request as soon
as its fixed step budget is done.  It reports solves per second and the
p50/p99 time from arrival to result.

The one-at-a-time baseline runs the same requests in FP64, each on its own
solver (create with the autotuned tile, run, read the diagnostics, destroy),
in arrival order.  Both build each request's initial fields on the device from
its closed-form shape (EULBFS_INIT_ANALYTIC).
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import List

import numpy as np

from . import eulbfs as E
from . import problems as PB

SIZES = (64, 128, 256, 512)
STATIC_SIGMA = PB.static_droplet()[0].sigma  # capillary number 0.01 of the 512 x 512 droplet


@dataclasses.dataclass
class Request:
    rid: int
    kind: str  # "static" or "impact"
    n: int
    nsteps: int
    draws: dict
    arrival: float = 0.0
    problem: object = None
    state: object = None


def draw_requests(count: int, seed: int = 0, nsteps: int = 2000, sizes=SIZES) -> List[Request]:
    """Seeded request mix: grid uniform over `sizes`, Ste ~ U[0.01, 1],
    supercooling ~ U[0.1, 1], contact angle ~ U[60, 120] deg, impact with
    probability 1/2 (We ~ U[5, 100], Re ~ U[100, 2000]); rho_s/rho_l = 0.917,
    gas/liquid density ratio 1/1000."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(rng.choice(sizes))
        d = dict(ste=float(rng.uniform(0.01, 1.0)), supercool=float(rng.uniform(0.1, 1.0)),
                 theta=float(rng.uniform(60.0, 120.0)))
        impact = bool(rng.random() < 0.5)
        if impact:
            d.update(we=float(rng.uniform(5.0, 100.0)), re=float(rng.uniform(100.0, 2000.0)))
        out.append(Request(rid=k, kind="impact" if impact else "static", n=n, nsteps=nsteps, draws=d))
    return out


def build(req: Request, precision: int):
    d = req.draws
    if req.kind == "impact":
        pr, st = PB.impact_droplet(n=req.n, we=d["we"], re=d["re"], ste=d["ste"], supercool=d["supercool"],
                                   theta_deg=d["theta"])
    else:
        pr, st = PB.static_droplet(n=req.n, R=req.n / 4, theta_deg=d["theta"], ste=d["ste"])
        pr = pr.replace(sigma=STATIC_SIGMA)
        st.T = np.where(st.C > 0.5, -d["supercool"], 0.0)
        st.shape = dataclasses.replace(st.shape, t_in=-d["supercool"])  # the same state, closed form
    return pr.replace(precision=precision), st


def poisson_arrivals(count: int, rate: float, seed: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count)) if rate > 0 else np.zeros(count)


def percentiles(lat):
    a = np.asarray(lat)
    return float(np.percentile(a, 50)), float(np.percentile(a, 99))


def serve(requests: List[Request], *, precision: int = E.FP32, hbm_budget: int = 2 << 30, max_slots: int = 64,
          tick_steps: int = 100, stream=None, tile: int = E.BATCH_TILE_AUTO) -> dict:
    """Run the requests through one batch; arrival times are in seconds from
    the start (requests[k].arrival).  Returns throughput and latency stats and
    the batch's tile choice (its measured device time per cell-step of each
    shape)."""
    import torch

    if stream is None:
        stream = torch.cuda.Stream()
    for r in requests:
        if r.problem is None:
            r.problem, r.state = build(r, precision)
    batch = E.Batch(hbm_budget, max_slots, precision=precision, stream=stream)
    batch.set_tile(tile)
    waiting = sorted(requests, key=lambda r: r.arrival)
    resident = {}  # slot -> request
    finish = {}
    admitted_at = {}
    failed = []
    t0 = time.perf_counter()
    ticks = 0
    enqueued = {}  # slot -> steps enqueued so far
    try:
        while waiting or resident:
            now = time.perf_counter() - t0
            # admit arrived requests, first come first served, while they fit
            while waiting and waiting[0].arrival <= now:
                r = waiting[0]
                slot = batch.admit(r.problem, r.state, r.nsteps, analytic=r.state.shape is not None)
                if slot is None:
                    break
                resident[slot] = r
                enqueued[slot] = 0
                admitted_at[r.rid] = time.perf_counter() - t0
                waiting.pop(0)
            if resident:
                left = [r.nsteps - enqueued[sl] for sl, r in resident.items() if enqueued[sl] < r.nsteps]
                if left:
                    step = min(tick_steps, min(left))  # the tick's common step count
                    batch.tick(tick_steps)
                    ticks += 1
                    for sl, r in resident.items():
                        if enqueued[sl] < r.nsteps:
                            enqueued[sl] += step
                else:
                    time.sleep(0.0005)  # everything resident is enqueued; wait for results
                for slot in batch.poll():
                    r = resident.pop(slot)
                    try:
                        d = batch.diagnostics(slot)
                        ok = d["nonfinite"] == 0 and d["steps"] == r.nsteps
                    except E.EulbfsError:  # the watchdog found the request unstable
                        ok = False
                    finish[r.rid] = time.perf_counter() - t0
                    if not ok:
                        failed.append(r.rid)
                    batch.release(slot)
                    enqueued.pop(slot, None)
            elif waiting:
                time.sleep(max(0.0, min(waiting[0].arrival - now, 0.05)))
        sched = batch.schedule()
    finally:
        batch.close()
    total = time.perf_counter() - t0
    lat = [finish[r.rid] - r.arrival for r in requests]
    p50, p99 = percentiles(lat)
    cells = sum(r.problem.cells * r.nsteps for r in requests)
    return {"solves": len(requests), "seconds": total, "solves_per_s": len(requests) / total,
            "p50_s": p50, "p99_s": p99, "mean_s": float(np.mean(lat)), "ticks": ticks,
            "cell_updates_per_s": cells / total, "failed": failed,
            "precision": "fp32" if precision == E.FP32 else "fp64", "tick_steps": tick_steps,
            "hbm_budget": hbm_budget, "max_slots": max_slots,
            "tile": {"mode": "auto" if tile == E.BATCH_TILE_AUTO else E.BATCH_TILE_NAMES[tile],
                     "next": E.BATCH_TILE_NAMES[sched["next_tile"]],
                     "ns_per_cell_step": {E.BATCH_TILE_NAMES[k + 1]: round(sched["ns_per_cell_step"][k], 5)
                                          for k in range(2)},
                     "ticks_timed": {E.BATCH_TILE_NAMES[k + 1]: sched["ticks_timed"][k] for k in range(2)},
                     "paired_time_ratio_64x8_over_32x16": round(sched["time_ratio"], 4),
                     "pairs": sched["pairs"]}}


def sequential(requests: List[Request], *, precision: int = E.FP64, stream=None) -> dict:
    """One request at a time on its own solver, in arrival order (arrivals are
    honoured: a request cannot start before it arrives)."""
    import torch

    if stream is None:
        stream = torch.cuda.Stream()
    order = sorted(requests, key=lambda q: q.arrival)
    built = [build(r, precision) for r in order]  # host-side inputs, outside the timed window as in serve()
    t0 = time.perf_counter()
    lat, failed = [], []
    cells = 0
    for r, (pr, st) in zip(order, built):
        now = time.perf_counter() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        s = E.Solver(pr, st, precision=precision, kernel=E.KERNEL_AUTO, stream=stream, analytic=st.shape is not None)
        try:
            s.step(r.nsteps)
            d = s.diagnostics()
            ok = d["nonfinite"] == 0
        except E.EulbfsError:  # the watchdog found the request unstable
            ok = False
        finally:
            s.close()
        if not ok:
            failed.append(r.rid)
        lat.append(time.perf_counter() - t0 - r.arrival)
        cells += pr.cells * r.nsteps
    total = time.perf_counter() - t0
    p50, p99 = percentiles(lat)
    return {"solves": len(requests), "seconds": total, "solves_per_s": len(requests) / total, "p50_s": p50,
            "p99_s": p99, "mean_s": float(np.mean(lat)), "cell_updates_per_s": cells / total, "failed": failed,
            "precision": "fp32" if precision == E.FP32 else "fp64"}


def accuracy(requests: List[Request], *, max_slots: int = 64, hbm_budget: int = 2 << 30, tick_steps: int = 100,
             stream=None) -> dict:
    """The served FP32 results against FP64: every request of the list runs
    through one FP32 batch (as served) and alone in FP64 (as the sequential
    baseline runs it); per request the relative L2 difference of each conserved
    field (H, p, the momentum vector, C) and the difference of the tip height
    and of the axis height (diagnostics 6 and 13), in cells."""
    import torch

    if stream is None:
        stream = torch.cuda.Stream()
    rows = []
    batch = E.Batch(hbm_budget, max_slots, precision=E.FP32, stream=stream)
    try:
        slots = {}
        for r in requests:
            pr, st = build(r, E.FP32)
            slot = batch.admit(pr, st, r.nsteps, analytic=st.shape is not None)
            if slot is None:
                raise RuntimeError("the accuracy subset must fit one batch")
            slots[r.rid] = slot
        nsteps = max(r.nsteps for r in requests)
        for _ in range((nsteps + tick_steps - 1) // tick_steps):
            batch.tick(tick_steps)
        stream.synchronize()
        assert len(batch.poll()) == len(requests)
        served = {rid: (batch.conserved(sl), batch.diagnostics(sl)) for rid, sl in slots.items()}
    finally:
        batch.close()
    for r in requests:
        pr, st = build(r, E.FP64)
        s = E.Solver(pr, st, precision=E.FP64, kernel=E.KERNEL_AUTO, stream=stream, analytic=st.shape is not None)
        try:
            s.step(r.nsteps)
            w64, d64 = s.conserved(), s.diagnostics()
        finally:
            s.close()
        w32, d32 = served[r.rid]
        err = {}
        for name, ks in (("H", [0]), ("p", [1]), ("M", [2, 3]), ("C", [4])):
            den = np.linalg.norm(w64[ks].ravel())
            err[name] = float(np.linalg.norm((w32[ks] - w64[ks]).ravel()) / den) if den > 0 else 0.0
        rows.append({"rid": r.rid, "n": r.n, "kind": r.kind, "rel_l2": err,
                     "tip_cells": abs(d32["tip"] - d64["tip"]) / pr.dx,
                     "axis_cells": abs(d32["axis_height"] - d64["axis_height"]) / pr.dx})
    worst = [max(row["rel_l2"].values()) for row in rows]
    fronts = [max(row["tip_cells"], row["axis_cells"]) for row in rows]
    return {"requests": len(rows), "steps_per_request": requests[0].nsteps if requests else 0,
            "rids": [row["rid"] for row in rows],
            "max_rel_l2": {k: max(row["rel_l2"][k] for row in rows) for k in ("H", "p", "M", "C")},
            "median_rel_l2": float(np.median(worst)), "max_front_cells": max(fronts),
            "median_front_cells": float(np.median(fronts)),
            "within_bar": bool(max(worst) <= 1e-4 and max(fronts) <= 0.5),
            "bar": "relative L2 <= 1e-4 per field, tip and axis heights within 0.5 cell"}


def run_mix(count: int = 256, nsteps: int = 2000, seed: int = 0, load: float = 0.8, hbm_budget: int = 2 << 30,
            max_slots: int = 64, tick_steps: int = 100, sizes=SIZES, with_sequential: bool = True,
            accuracy_requests: int = 24, compare_tiles: bool = True) -> dict:
    """The serving benchmark: (1) all requests at t = 0 through the batched
    FP32 server (capacity) with the tile chosen on the fly, and (with
    compare_tiles) again with each tile shape pinned, (2) Poisson arrivals at
    `load` times that capacity (latency under load), (3) the sequential FP64
    baseline on the burst."""
    reqs = draw_requests(count, seed=seed, nsteps=nsteps, sizes=sizes)
    burst = serve(reqs, hbm_budget=hbm_budget, max_slots=max_slots, tick_steps=tick_steps)
    pinned = {}
    if compare_tiles:
        for tile, name in E.BATCH_TILE_NAMES.items():
            rp = draw_requests(count, seed=seed, nsteps=nsteps, sizes=sizes)
            pinned[name] = round(serve(rp, hbm_budget=hbm_budget, max_slots=max_slots, tick_steps=tick_steps,
                                       tile=tile)["solves_per_s"], 2)
    rate = load * burst["solves_per_s"]
    arr = poisson_arrivals(count, rate, seed=seed + 1)
    reqs2 = draw_requests(count, seed=seed, nsteps=nsteps, sizes=sizes)
    for r, a in zip(reqs2, arr):
        r.arrival = float(a)
    loaded = serve(reqs2, hbm_budget=hbm_budget, max_slots=max_slots, tick_steps=tick_steps)
    out = {"requests": count, "steps_per_request": nsteps, "seed": seed, "batched_fp32_burst": burst,
           "batched_fp32_poisson": dict(loaded, arrival_rate_per_s=rate, load=load)}
    if pinned:
        out["batched_fp32_burst_pinned_tile_solves_per_s"] = pinned
    if with_sequential:
        reqs3 = draw_requests(count, seed=seed, nsteps=nsteps, sizes=sizes)
        out["sequential_fp64_burst"] = sequential(reqs3)
        out["speedup_solves_per_s"] = burst["solves_per_s"] / out["sequential_fp64_burst"]["solves_per_s"]
    if accuracy_requests:
        # every (count // accuracy_requests)-th request of the mix
        reqs4 = draw_requests(count, seed=seed, nsteps=nsteps, sizes=sizes)
        step = max(1, count // accuracy_requests)
        out["accuracy_fp32_vs_fp64"] = accuracy(reqs4[::step][:accuracy_requests], max_slots=max_slots,
                                                hbm_budget=hbm_budget, tick_steps=tick_steps)
    return out


if __name__ == "__main__":
    import json
    import sys

    n = int(sys.argv[1]) if len(sys.argv) > 1 else 256
    print(json.dumps(run_mix(count=n)), flush=True)
