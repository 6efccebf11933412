#!/usr/bin/env python3
"""Benchmark of the EULBFS time step on one MI355X.

Workload: the static-droplet freezing problem of Sec. 3.4 at 512 x 512 cells
(droplet radius 128 on a cold wall, contact angle 90 deg, rho_s/rho_l = 0.917,
gas/liquid density ratio 1/1000, Ste = 0.1, Ca = 0.01), synthetic initial
state, FP64, fused flux + update kernel.  One step = one SSP-RK3 time step
(three fused stage launches) over the whole grid.

Prints one JSON line: cell updates per second (MLUPS); the roofline of the
fused stage kernel (counted flop per launch over its average launch time,
measured with HIP events on the stream the kernels run on, with the
algorithmic HBM bytes per launch beside it); the continuous-batching serving
mix (solves/s, p50/p99 time to solution, against one-at-a-time FP64); and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s (MLUPS) & % HBM BW; batched solves/s + p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# Published vector peaks of MI355X (256 CUs at 2.4 GHz): FP64 78.6 TFLOP/s,
# FP32 157.3 TFLOP/s.  The FP32 figure assumes packed FP32 issue; the kernels
# are built with packed FP32 off, so for them it is an upper bound.
VALU_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
# Per tile shape of k_stage_fused on the 512 x 512 droplet, counted with
# rocprofv3 (profiles/k_stage_fused_droplet512.md):
#   f64 / f32  floating-point operations per cell and RK stage executed
#              (SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64 / _F32, 64 lanes per
#              wave instruction, FMA = 2; they include the tile's recomputed
#              halo of primitives and faces); the FP32 mode still does the
#              closure, the H and C combination and mu_c in FP64
#   valu       VALU lane-instructions per cell and stage (SQ_INSTS_VALU x 64)
#   hbm        HBM bytes per launch: FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (KiB
#              per dispatch; the factors make a 1 GiB device copy read and
#              write 1 GiB)
# valid only for the sources and compile flags with this fingerprint (sha256
# of csrc/eulbfs_device.h, csrc/eulbfs_internal.h, csrc/eulbfs_kernels.hip and
# build.py).
COUNTS_FINGERPRINT = "faa2f891ed7b98a2"
COUNTS = {
    "fp64/32x8": {"f64": 1138.7, "valu": 1103.0, "hbm": 31888981},
    "fp64/64x4": {"f64": 1159.3, "valu": 1149.5, "hbm": 31880789},
    "fp64/16x16": {"f64": 1139.0, "valu": 1095.8, "hbm": 31874648},
    "fp64/64x8": {"f64": 1038.9, "valu": 1016.6, "hbm": 31870549},
    "fp64/32x16": {"f64": 1033.5, "valu": 1000.3, "hbm": 31871830},
    "fp64/32x32": {"f64": 1024.8, "valu": 989.6, "hbm": 31918462},
    "fp32/32x8": {"f32": 1060.3, "f64": 61.4, "valu": 1137.8, "hbm": 21818933},
    "fp32/64x4": {"f32": 1064.9, "f64": 73.5, "valu": 1186.1, "hbm": 21826072},
    "fp32/16x16": {"f32": 1060.3, "f64": 61.7, "valu": 1127.8, "hbm": 22437606},
    "fp32/64x8": {"f32": 964.4, "f64": 59.0, "valu": 1048.1, "hbm": 21810918},
    "fp32/32x16": {"f32": 963.3, "f64": 55.7, "valu": 1029.9, "hbm": 21807684},
    "fp32/32x32": {"f32": 913.2, "f64": 51.6, "valu": 974.9, "hbm": 21845504},
}
# an FP64 VALU instruction of a wave64 occupies its 16-lane SIMD for 4 cycles:
# 1024 SIMDs x 2.4 GHz / 4 wave-instructions per second.  Other VALU
# instructions can issue faster (the FP32 kernel exceeds this rate on a
# 4096 x 4096 grid), so for the FP32 mode the fraction overstates the load.
VALU_ISSUE_PEAK = 1024 * 2.4e9 / 4


def flop_peak(mix: dict):
    """Counted flop per cell and stage, and the peak for that mix of FP32 and
    FP64 operations (time at peak of each part, summed)."""
    parts = {k: v for k, v in mix.items() if k in VALU_PEAK_TFLOPS}
    flop = sum(parts.values())
    return flop, flop / sum(v / VALU_PEAK_TFLOPS[k] for k, v in parts.items())


# compulsory HBM words per cell and time step (SSP-RK3 over the five conserved
# planes and the dF_s/dt plane): stage 1 reads W^n and dF_s/dt and writes W1
# (11), stage 2 reads W1, W^n, dF_s/dt and writes W2 (16), stage 3 reads W2,
# W^n, dF_s/dt and writes W^{n+1} and dF_s/dt (17)
WORDS_PER_CELL_STEP = 44


def bytes_per_cell_step(precision: int) -> int:
    if precision == 0:
        return WORDS_PER_CELL_STEP * 8
    # FP32 mode keeps H and C in FP64: per copy of W 2 x 8 + 3 x 4 bytes, eight
    # copies moved per step, plus four transfers of the FP32 dF_s/dt plane
    return 8 * (2 * 8 + 3 * 4) + 4 * 4


def kernel_fingerprint() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in ("csrc/eulbfs_device.h", "csrc/eulbfs_internal.h", "csrc/eulbfs_kernels.hip",
              "build.py"):  # sources and compile flags
        with open(os.path.join(ROOT, "paper_2507_03366_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload(name: str):
    from paper_2507_03366_amd import problems as PB

    if name == "C4":
        pr, st = PB.static_droplet()
        desc = ("static droplet freezing on a cold wall, 512x512 cells, R=128, theta=90deg, rho_s/rho_l=0.917, "
                "rho_g/rho_l=1e-3, Ste=0.1, Ca=0.01")
    elif name == "C1":
        pr, st = PB.conductive_freezing()
        desc = "conductive freezing (one-phase Neumann), 128x4 cells, Ste=0.1, alpha=0.4"
    elif name == "C3":
        pr, st = PB.film_freezing()
        desc = "liquid film freezing, 256x256 cells, film height 0.3, Bo=1, Ste=0.05, rho_s/rho_l=0.917"
    elif name == "C2":
        pr, st = PB.three_phase_stefan()
        desc = "three-phase Stefan problem, 256x8 cells, rho_s/rho_l=0.9, rho_g/rho_l=1e-3, Ste=0.1"
    elif name == "G512":
        pr, st = PB.static_droplet()
        wy = PB.graded_widths(pr.ny, 0.5, 1.02, 1.0)
        pr = pr.replace(y_width=wy, delta_t=0.25, dt=0.25)
        X, Y = PB.cell_centres(pr)
        st.C = PB.droplet_profile(X, Y, 0.5 * pr.nx, 0.0, 128.0, pr.xi)
        desc = ("static droplet freezing on a cold wall, 512x512 cells on a stretched mesh (rows from 0.5 at the "
                "wall growing 2 % per row to 1.0), R=128, theta=90deg, rho_s/rho_l=0.917, rho_g/rho_l=1e-3, "
                "Ste=0.1, Ca=0.01, delta_t = dt = 0.25")
    elif name.startswith("R"):
        n = int(name[1:])
        pr, st = PB.static_droplet(n=n, R=n / 4)
        pr = pr.replace(sigma=PB.static_droplet()[0].sigma)
        desc = f"static droplet freezing scaled to {n}x{n} cells (R={n // 4}), same material constants as 512x512"
    else:
        raise SystemExit(f"unknown workload {name}")
    return pr, st, desc


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_rate(pr, st, budget_s: float, threads: int):
    """Oracle steps of the workload from its initial state for about budget_s
    seconds on `threads` threads: (MLUPS, steps, seconds)."""
    from oracle import oracle as O
    import numpy as np

    O.set_threads(threads)
    W = O.init(pr, st)
    fs = np.zeros((pr.ny, pr.nx))
    t0 = time.perf_counter()
    W, fs = O.step(pr, W, fs, 1)  # the first step also starts the thread pool
    t1 = time.perf_counter()
    W, fs = O.step(pr, W, fs, 1)
    t2 = time.perf_counter()
    steps = 2
    more = int(max(0.0, budget_s - (t2 - t0)) / max(t2 - t1, 1e-6))
    if more > 0:
        W, fs = O.step(pr, W, fs, more)
        steps += more
    el = time.perf_counter() - t0
    return pr.cells * steps / el / 1e6, steps, el


def cpu_baseline(pr, st, budget_s: float):
    """Time the FP64 oracle as it stands (gcc -O3, OpenMP over rows) on this
    host's cores, and on one thread."""
    from oracle import oracle as O

    O.build(force=False)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    mlups, steps, el = oracle_rate(pr, st, budget_s, threads)
    used = O.num_threads()
    one, steps1, el1 = oracle_rate(pr, st, budget_s / 3.0, 1)
    O.set_threads(threads)
    return {"value": mlups, "unit": "MLUPS", "cores": used, "kind": "oracle",
            "sample": f"{steps} oracle steps of the same {pr.nx}x{pr.ny} workload from its initial state, "
                      f"{el:.1f} s wall on {used} threads",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "one_thread": {"value": one, "unit": "MLUPS", "sample": f"{steps1} steps, {el1:.1f} s wall"}}


def hbm_point(name: str, precision: int, steps: int):
    """A single large grid: MLUPS and compulsory HBM bytes per second of the
    autotuned fused kernel (HIP events on the solver's stream)."""
    import torch
    from paper_2507_03366_amd import eulbfs as E

    pr, st, _ = workload(name)
    stream = torch.cuda.Stream()
    s = E.Solver(pr, st, precision=precision, kernel=E.KERNEL_AUTO, stream=stream, analytic=True)
    try:
        sched = s.schedule()
        s.step(8)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        finite = s.diagnostics()["nonfinite"] == 0
    finally:
        s.close()
    bpcs = bytes_per_cell_step(precision)
    rate = pr.cells * steps / (ms * 1e-3)
    ws = pr.cells * (bpcs / 44.0 * 16)  # W^n, two RK registers and dF_s/dt, bytes
    return {"workload": f"{pr.nx}x{pr.ny}", "precision": "fp64" if precision == 0 else "fp32",
            "tile": f"{sched[1]}x{sched[2]}", "steps": steps, "ms_per_step": round(ms / steps, 5),
            "mlups": round(rate / 1e6, 1), "bytes_per_cell_step": bpcs,
            "gbs": round(rate * bpcs / 1e9, 1), "frac": round(rate * bpcs / 1e9 / HBM_PEAK_GBS, 4),
            "working_set_mb": round(ws / 1e6, 1), "finite": bool(finite)}


def hbm_batch_point(count: int, n: int, steps: int):
    """count droplets of n x n in one FP32 batch, advanced by ticks of `steps`
    steps: MLUPS and compulsory HBM bytes per second of the batched kernel."""
    import torch
    from paper_2507_03366_amd import eulbfs as E
    from paper_2507_03366_amd import problems as PB

    pr, st = PB.static_droplet(n=n, R=n / 4)
    pr = pr.replace(sigma=PB.static_droplet()[0].sigma, precision=1)
    need = E.eulbfs_batch_request_bytes(E.params_from_problem(pr, precision=E.FP32))
    stream = torch.cuda.Stream()
    b = E.Batch(need * count + (64 << 20), count, precision=E.FP32, stream=stream)
    b.set_tile(E.BATCH_TILE_32x16)  # the shape a batch settles on for the serving mix
    try:
        for _ in range(count):
            assert b.admit(pr, st, 2 * steps + 8) is not None
        b.tick(8)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.tick(steps)
        b.tick(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
    finally:
        b.close()
    bpcs = bytes_per_cell_step(1)
    rate = count * pr.cells * 2 * steps / (ms * 1e-3)
    return {"workload": f"{count} x {n}x{n} batch", "precision": "fp32", "tile": "32x16", "steps": 2 * steps,
            "ms_per_step": round(ms / (2 * steps), 5), "mlups": round(rate / 1e6, 1), "bytes_per_cell_step": bpcs,
            "gbs": round(rate * bpcs / 1e9, 1), "frac": round(rate * bpcs / 1e9 / HBM_PEAK_GBS, 4),
            "working_set_mb": round(count * need / 1e6, 1)}


# Per-config windows: (workload, oracle steps on all cores, oracle steps on
# one thread, steps to the configuration's end point or None).  C1 and C2 run
# their full length on all cores; C3 and C4 a 1000-step window, whose
# time to solution is extrapolated and labelled so.
CONFIG_WINDOWS = (("C1", 20000, 20000, 20000), ("C2", 50000, 2000, 50000), ("C3", 1000, 100, 360000),
                  ("C4", 1000, 100, None))


def gpu_rate(pr, st, precision: int, steps: int):
    """MLUPS of the autotuned fused kernel over `steps` steps (HIP events on
    the solver's stream) and the seconds they took."""
    import torch
    from paper_2507_03366_amd import eulbfs as E

    stream = torch.cuda.Stream()
    s = E.Solver(pr, st, precision=precision, kernel=E.KERNEL_AUTO, stream=stream)
    try:
        s.step(8)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3
    finally:
        s.close()
    return pr.cells * steps / sec / 1e6, sec


def config_table():
    """The oracle (all cores and one thread) and the GPU path (FP64 and FP32
    mode) on each configuration's window."""
    from oracle import oracle as O

    O.build(force=False)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rows = []
    for name, n_all, n_one, n_end in CONFIG_WINDOWS:
        pr, st, desc = workload(name)
        row = {"config": name, "workload": desc, "cells": pr.cells}
        O.set_threads(threads)
        t0 = time.perf_counter()
        O.run(pr, st, n_all)
        el = time.perf_counter() - t0
        row["oracle_all_cores"] = {"steps": n_all, "seconds": round(el, 2), "threads": O.num_threads(),
                                   "mlups": round(pr.cells * n_all / el / 1e6, 3)}
        O.set_threads(1)
        t0 = time.perf_counter()
        O.run(pr, st, n_one)
        el1 = time.perf_counter() - t0
        row["oracle_one_thread"] = {"steps": n_one, "seconds": round(el1, 2),
                                    "mlups": round(pr.cells * n_one / el1 / 1e6, 3)}
        g64, s64 = gpu_rate(pr, st, 0, n_all)
        g32, s32 = gpu_rate(pr, st, 1, n_all)
        row["gpu_fp64"] = {"steps": n_all, "seconds": round(s64, 4), "mlups": round(g64, 1)}
        row["gpu_fp32"] = {"steps": n_all, "seconds": round(s32, 4), "mlups": round(g32, 1)}
        if n_end:
            tag = "measured" if n_end == n_all else f"extrapolated from the {n_all}-step window"
            row["time_to_solution_s"] = {"steps": n_end, "oracle_all_cores": round(n_end * el / n_all, 1),
                                         "gpu_fp64": round(n_end * s64 / n_all, 3),
                                         "gpu_fp32": round(n_end * s32 / n_all, 3), "how": tag}
        rows.append(row)
        print(json.dumps(row), flush=True)
    O.set_threads(threads)
    return {"cpu_model": cpu_model(), "nproc": os.cpu_count(), "configs": rows}


def hbm_sweep():
    """The droplet scaled to 1024^2, 2048^2 and 4096^2 in FP64 and FP32 mode
    (the working set passes the 256 MB Infinity Cache between 1024^2 and
    2048^2), and 64 droplets of 512^2 in one FP32 batch."""
    pts = []
    for n, steps in ((1024, 200), (2048, 100), (4096, 60)):
        pts += [hbm_point(f"R{n}", 0, steps), hbm_point(f"R{n}", 1, steps)]
    return pts + [hbm_batch_point(64, 512, 30)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=192)
    ap.add_argument("--warmup", type=int, default=32)
    ap.add_argument("--workload", default="C4")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--kernel", default="auto", choices=["auto", "fused", "split"],
                    help="auto: the library times every tile shape of the fused kernel at create")
    ap.add_argument("--tile", default="0x0")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serving", type=int, default=256, metavar="REQUESTS",
                    help="requests of the continuous-batching serving mix (0: skip)")
    ap.add_argument("--serving-steps", type=int, default=2000)
    ap.add_argument("--no-hbm-sweep", action="store_true",
                    help="skip the large-grid points whose working set exceeds the 256 MB Infinity Cache")
    ap.add_argument("--only-hbm-sweep", action="store_true",
                    help="run only the large-grid points and print them (for profiling them alone)")
    ap.add_argument("--config-table", action="store_true",
                    help="only time the oracle and the GPU path on each configuration's window")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); a multi-GPU run is not part of this build",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2507_03366_amd import eulbfs as E

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 8, "launches": 5}), flush=True)
        return
    if args.config_table:
        print(json.dumps(config_table()), flush=True)
        return
    if args.only_hbm_sweep:
        print(json.dumps({"hbm_sweep": hbm_sweep()}), flush=True)
        return
    pr, st, desc = workload(args.workload)
    precision = 0 if args.precision == "fp64" else 1
    kernel = {"auto": E.KERNEL_AUTO, "fused": E.KERNEL_FUSED, "split": E.KERNEL_SPLIT}[args.kernel]
    tile = tuple(int(v) for v in args.tile.split("x"))
    # a created stream: the solver captures its steps into a HIP graph and replays it
    stream = torch.cuda.Stream()
    s = E.Solver(pr, st, precision=precision, kernel=kernel, tile=tile, stream=stream)
    sched = s.schedule()
    s.step(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    diag = s.diagnostics()
    s.close()
    if diag["nonfinite"] != 0:
        raise SystemExit("state became non-finite during the benchmark")
    # the same steps with the host hand-over included: create from host planes
    # (upload), step, read the conserved state back (download); not `value`
    t0 = time.perf_counter()
    s = E.Solver(pr, st, precision=precision, kernel=E.KERNEL_SPLIT if sched[0] == E.KERNEL_SPLIT else E.KERNEL_FUSED,
                 tile=(sched[1], sched[2]), stream=stream)
    s.step(args.steps)
    s.conserved()
    pcie_s = time.perf_counter() - t0
    s.close()

    cells = pr.cells
    mlups = cells * args.steps / (ms * 1e-3) / 1e6
    # one launch of the dominant kernel per RK stage (split: four kernels per stage)
    kname = "k_stage_fused" if sched[0] == E.KERNEL_FUSED else "split stage (4 kernels)"
    launches = 3 * args.steps
    avg_launch_us = ms * 1e3 / launches
    bpcs = bytes_per_cell_step(precision)
    alg_bytes_per_launch = bpcs * cells / 3.0
    hbm_gbs = alg_bytes_per_launch / (avg_launch_us * 1e-6) / 1e9
    fp = kernel_fingerprint()
    ckey = f"{args.precision}/{sched[1]}x{sched[2]}"
    uniform = pr.x_width is None and pr.y_width is None  # the counts are of the uniform-mesh kernels
    counts = COUNTS.get(ckey) if (fp == COUNTS_FINGERPRINT and sched[0] == E.KERNEL_FUSED and uniform) else None
    if counts:
        flop_cell, peak_tflops = flop_peak(counts)
        flop_per_launch = flop_cell * cells
        tflops = flop_per_launch / (avg_launch_us * 1e-6) / 1e12
        issue = counts["valu"] / 64 * cells / (avg_launch_us * 1e-6) / VALU_ISSUE_PEAK
    else:  # the counters were taken on other kernel sources or another kernel (or mesh kind)
        flop_cell = peak_tflops = flop_per_launch = tflops = issue = None
    traffic = counts["hbm"] if (counts and args.workload == "C4") else None
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == 0 else "f32 (H, C in f64)",
        "data": "synthetic",
        "config": {"workload": desc, "nx": pr.nx, "ny": pr.ny, "precision": args.precision,
                   "kernel": args.kernel, "tile": args.tile, "steps_are": "SSP-RK3 time steps",
                   "schedule": {"kernel": {0: "fused", 1: "split"}[sched[0]],
                                "tile": f"{sched[1]}x{sched[2]}"}},
        # the binding roof is the vector ALU: the kernel's ~10 counted FP64 flop
        # per compulsory HBM byte sits at the FP64 ridge (78.6 TFLOP/s over
        # 8 TB/s = 9.8), and every VALU instruction, FP64 or not, holds its
        # SIMD for 4 cycles; the HBM view is given beside it
        "roofline": {"bound": "alu", "achieved": tflops and round(tflops, 2),
                     "peak": peak_tflops and round(peak_tflops, 1), "unit": "TFLOP/s",
                     "frac": tflops and round(tflops / peak_tflops, 4), "traffic": traffic,
                     "kernel": kname, "tile": f"{sched[1]}x{sched[2]}", "avg_launch_us": round(avg_launch_us, 2),
                     "flop_per_cell_stage": counts and {k: v for k, v in counts.items() if k in VALU_PEAK_TFLOPS},
                     "alg_flop_per_launch": flop_per_launch and int(flop_per_launch),
                     "valu_issue_frac": issue and round(issue, 4),
                     "kernel_fingerprint": fp,
                     "hbm": {"achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(hbm_gbs / HBM_PEAK_GBS, 4),
                             "alg_bytes_per_launch": int(alg_bytes_per_launch), "bytes_per_cell_step": bpcs}},
        "host_handover": {"mlups": round(pr.cells * args.steps / pcie_s / 1e6, 2), "seconds": round(pcie_s, 4),
                          "what": "create from host planes + the timed steps + W read back to the host"},
        "diagnostics_after": {k: float(v) for k, v in diag.items()},
    }
    if not args.no_hbm_sweep:
        # the 512 x 512 state (34 MB) lives in the 256 MB Infinity Cache: the
        # HBM fraction is measured on working sets well beyond it
        out["hbm_sweep"] = hbm_sweep()
    if args.serving:
        from paper_2507_03366_amd import serve as S

        out["serving"] = S.run_mix(count=args.serving, nsteps=args.serving_steps,
                                   accuracy_requests=min(24, args.serving))
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(pr, st, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
