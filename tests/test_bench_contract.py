"""The benchmark's command-line contract: one GPU only, and one JSON line
with the fields the measurement needs (roofline and the oracle baseline
included)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")

sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_lookup_counts():
    # 16 lookups per round; CTR shares 12 of round 1's between all blocks
    assert bench.lookups_per_block(10) == 160
    assert bench.lookups_per_block(14) == 224
    assert bench.lookups_per_block(10, ctr=True) == 148


def test_launch_stats_drops_outliers_like_the_paper():
    t = [1e-3] * 9 + [5e-3]
    s = bench.launch_stats(t)
    assert s["launches"] == 10 and s["kept"] == 9
    assert s["median"] == 1000.0 and s["max"] == 5000.0
    assert s["paper_style_mean"] == 1000.0
    assert s["mean"] == pytest.approx(1400.0)


@pytest.mark.gpu
def test_bench_line_fields():
    cmd = [sys.executable, "-u", BENCH, "--steps", "3", "--warmup", "1", "--nbytes", str(16 << 20),
           "--cpu-sample-mib", "1", "--no-secondary", "--no-batched", "--no-served", "--no-sweep"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1
    assert d["value"] > 0 and d["higher_is_better"] is True and d["vs_baseline"] is None
    assert d["dtype"] == "u8" and "workload" in d["config"]
    roof = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in roof, k
    assert roof["frac"] == pytest.approx(roof["achieved"] / roof["peak"], rel=1e-3)
    cpu = d["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["value"] > 0 and cpu["cores"] >= 1 and cpu["sample"]
    assert "cpu_context" in d and (d["cpu_context"] is None or d["cpu_context"]["GB/s"] > 0)
    lds = d["lds_gather"]
    assert lds["Tlookup/s"] > 0 and d["roofline_issue"]["measured_peak"] == lds["Tlookup/s"]


def test_cpu_baseline_record():
    # the oracle on a 1 MiB sample: all cores and one thread, one warm-up and
    # the median of five runs each, with the host's CPU model
    c = bench.cpu_baseline(1 << 20)
    assert c["kind"] == "oracle" and c["unit"] == "GB/s" and c["value"] > 0
    assert c["cores"] == len(os.sched_getaffinity(0))
    assert c["cpu_model"] is None or len(c["cpu_model"]) > 3
    assert "median of 5 runs" in c["sample"] and "warm-up" in c["sample"]
    assert c["single_thread_GB/s"] > 0 and "median of 5 runs" in c["single_thread_sample"]
    assert c["paper_style_GB/s"] > 0


def test_cpu_context_record():
    # openssl speed for context, kept apart from the oracle baseline; absent
    # (None) only where the host has no openssl executable
    import shutil
    c = bench.cpu_context_openssl()
    if shutil.which("openssl") is None:
        assert c is None
        return
    assert c["GB/s"] > 0 and c["processes"] == len(os.sched_getaffinity(0))
    assert c["kind"].startswith("openssl speed") and "aes-128-ecb" in c["command"]
