"""bench.py keeps its output contract: one JSON line with the metric, the
roofline and (on request) the serving and CPU-baseline objects; more than
one GPU is refused with a message."""
import json
import pathlib
import subprocess
import sys

import pytest

ROOT = pathlib.Path(__file__).resolve().parent.parent


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.gpu
def test_bench_json_line():
    r = subprocess.run([sys.executable, "-u", str(ROOT / "bench.py"), "--steps", "3", "--warmup", "1",
                        "--serving", "6", "--serving-steps", "20", "--cpu-budget", "1"],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "serving", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["value"] > 0
    assert d["config"]["workload"].startswith("static droplet")
    rl = d["roofline"]
    assert rl["bound"] == "alu" and rl["avg_launch_us"] > 0 and 0 < rl["hbm"]["frac"] < 1
    if rl["frac"] is not None:
        assert 0 < rl["frac"] < 1 and 0 < rl["valu_issue_frac"] < 1
    assert d["serving"]["batched_fp32_burst"]["failed"] == []
    assert set(d["serving"]["batched_fp32_burst_pinned_tile_solves_per_s"]) == {"32x16", "64x8"}
    assert d["serving"]["batched_fp32_burst"]["tile"]["mode"] == "auto"
    acc = d["serving"]["accuracy_fp32_vs_fp64"]
    assert acc["requests"] == 6 and acc["within_bar"], acc
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0
    assert cb["one_thread"]["value"] > 0 and cb["cpu_model"]
    sweep = d["hbm_sweep"]
    assert [p["workload"] for p in sweep] == ["1024x1024", "1024x1024", "2048x2048", "2048x2048", "4096x4096",
                                              "4096x4096", "64 x 512x512 batch"]
    for p in sweep:
        assert 0 < p["frac"] < 1 and p["mlups"] > 0
        if p["workload"] in ("4096x4096", "64 x 512x512 batch"):
            assert p["working_set_mb"] > 1000  # far beyond the 256 MB Infinity Cache


@pytest.mark.gpu
def test_bench_stretched_workload():
    """The graded-mesh droplet runs through the same contract (fused 32x16
    tiles, a CPU baseline from the oracle on the same stretched mesh)."""
    r = subprocess.run([sys.executable, "-u", str(ROOT / "bench.py"), "--workload", "G512", "--steps", "3",
                        "--warmup", "1", "--serving", "0", "--cpu-budget", "1", "--no-hbm-sweep"],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    assert "stretched mesh" in d["config"]["workload"] and d["value"] > 0
    assert d["config"]["schedule"] == {"kernel": "fused", "tile": "32x16"}
    assert d["diagnostics_after"]["nonfinite"] == 0
    # the counted operations are of the uniform-mesh kernel: none for this one
    assert d["roofline"]["flop_per_cell_stage"] is None and d["roofline"]["traffic"] is None
    assert d["cpu_baseline"]["value"] > 0
