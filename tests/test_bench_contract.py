"""The benchmark's command-line contract: one JSON line with the metric, the whole-job
value, the timing fields, the roofline of the dominant kernel and the oracle's CPU
baseline; more than one GPU is refused before any GPU work."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    run = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                         capture_output=True, text=True, timeout=120)
    assert run.returncode == 2
    assert "one GPU" in run.stderr and run.stdout == ""


@pytest.mark.gpu
@pytest.mark.timeout(600)
def test_bench_prints_one_json_line():
    run = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--workload", "scattering", "--n",
                          "32", "--steps", "2", "--warmup", "1", "--cpu-sweeps", "1"], cwd=ROOT, capture_output=True,
                         text=True, timeout=500)
    assert run.returncode == 0, run.stderr[-3000:]
    lines = [l for l in run.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    out = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in out, key
    assert out["n_gpus"] == 1 and out["steps"] == 2 and out["warmup"] == 1
    assert out["value"] > 0 and out["ms_per_step"] > 0 and out["higher_is_better"] is True
    assert "workload" in out["config"] and out["vs_baseline"] is None
    r = out["roofline"]
    assert r["bound"] == "alu" and r["unit"] == "Tops/s" and 0 < r["frac"] < 1
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-12
    assert r["traffic"] is None   # byte counters were taken on the 128^3 workload only
    c = out["cpu_baseline"]
    assert c["kind"] == "oracle" and c["cores"] == 1 and c["value"] > 0 and c["sample"]


@pytest.mark.gpu
@pytest.mark.timeout(600)
def test_bench_default_multifreq_line():
    """The default line (multi-frequency workload, here on a small grid and 4 bins): one
    JSON line whose roofline carries the VALU and the HBM fractions, the 128^3 scattering
    solves beside it (here 32^3), and a CPU baseline with its single-thread leg."""
    run = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--mf-n", "32", "--bins", "4",
                          "--steps", "3", "--warmup", "1", "--n", "32", "--scattering-steps", "1"], cwd=ROOT,
                         capture_output=True, text=True, timeout=500)
    assert run.returncode == 0, run.stderr[-3000:]
    lines = [l for l in run.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    out = json.loads(lines[0])
    assert out["steps"] == 3 and out["warmup"] == 1 and out["value"] > 0
    assert out["config"]["bins"] == 4 and out["config"]["rays"] == 80
    r = out["roofline"]
    assert r["bound"] == "alu" and 0 < r["frac"] < 1 and r["traffic"] is None
    h = r["hbm"]
    assert h["unit"] == "GB/s" and abs(h["frac"] - h["achieved"] / h["peak"]) < 1e-12
    assert abs(h["bytes_per_update"] - 1.2) < 1e-12
    assert out["scattering_128"]["ali_solves_per_s"] > 0
    c = out["cpu_baseline"]
    assert c["kind"] == "oracle" and c["cores"] >= 1 and c["value"] > 0
    assert c["single_thread"]["cores"] == 1 and c["single_thread"]["value"] > 0


@pytest.mark.gpu
@pytest.mark.timeout(600)
def test_bench_serving_line():
    """The serving workload at a reduced request size and window: one JSON line with the
    overload figure, the capacity and the latency curve."""
    run = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--workload", "serving",
                          "--serve-window", "3", "--streams", "2", "--serve-max-n", "40"],
                         cwd=ROOT, capture_output=True, text=True, timeout=500)
    assert run.returncode == 0, run.stderr[-3000:]
    lines = [l for l in run.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    out = json.loads(lines[0])
    assert out["unit"] == "solves/s" and out["value"] > 0 and out["capacity_solves_per_s"] > 0
    assert [round(r["rate_per_s"] / out["capacity_solves_per_s"], 2) for r in out["latency_vs_rate"]] == \
        [0.25, 0.5, 0.9]
    for r in out["latency_vs_rate"] + [out["overload_200_per_s"]]:
        assert r["served"] + r["unserved"] == r["arrived"]
        if r["served"]:
            assert 0 < r["latency_ms"]["p50"] <= r["latency_ms"]["p99"]
        assert r["not_converged"] == 0
    assert out["overload_200_per_s"]["arrived"] > 0
