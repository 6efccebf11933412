"""Sec. 3.5 on the GPU: a water droplet (case (b) of the text) impacting a cold
wall on the paper's 400 x 200 grid, with the spreading diameter D (wetted
length on the wall) and the bounce height H_b (condensed height on the axis)
of the diagnostics query.

Measured against Tables 6-7: the largest spreading factor within 10 % of the
paper's simulated 1.61 (this build: 1.52; the experiment's 1.55), the largest
spread shrinking as the wall gets colder (Fig. 18) and the bounce height at
15 ms growing as it does (Table 7's trend; the values themselves come out
higher here, 0.82-0.95 against 0.62-0.68).  The runs stop at the first
non-finite state (the watchdog).  Case (a), the higher Weber and Reynolds
numbers, is not run: its gas, squeezed from under the drop, exceeds the
lattice sound speed within a few hundred steps at any lattice impact speed
and resolution tried.
"""
import os

import numpy as np
import pytest

from paper_2507_03366_amd import eulbfs as E
from paper_2507_03366_amd import problems as PB

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    out = {}
    with open(os.path.join(HERE, "golden", "impact_sec35.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split("=")
                out[k.strip()] = [float(x) for x in v.split()]
    return out


G = _golden()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    E.lib()
    yield


def _history(T_w, t_end, every=200):
    import torch

    pr, st = PB.impact_sec35("b", T_w=T_w)
    s = E.Solver(pr, st, kernel=E.KERNEL_AUTO, stream=torch.cuda.Stream(), analytic=True)
    hist = []
    try:
        n = int(np.ceil(t_end / pr.dt))
        done = 0
        while done < n:
            k = min(every, n - done)
            s.run(k)
            done += k
            d = s.diagnostics()
            hist.append((d["time"], d["wetted_length"] / 100.0, d["axis_height"] / 100.0))
    finally:
        s.close()
    return hist


def test_spreading_and_bounce_against_tables_6_and_7():
    t15 = PB.impact_time("b", 0.015)
    spread, bounce = {}, {}
    for T_w in G["table7_T_w"]:
        h = _history(T_w, t15)
        spread[T_w] = max(x[1] for x in h)
        bounce[T_w] = h[-1][2]
    print({T_w: (round(spread[T_w], 3), round(bounce[T_w], 3)) for T_w in spread}, "Table 7",
          G["table7_H_b_over_D_0"])
    ws = G["table7_T_w"]  # -20, -25, -30, -35: colder to the right
    assert abs(spread[-30.0] / G["table6_simulation"][1] - 1.0) < 0.10
    assert all(spread[a] > spread[b] for a, b in zip(ws, ws[1:]))
    assert all(bounce[a] < bounce[b] for a, b in zip(ws, ws[1:]))
