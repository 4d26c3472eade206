"""bench.py keeps its output contract: one JSON line with the keys the
result is read by, a refusal of several GPUs, and a traffic figure only
while the committed counter summary matches the sweep's sources."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KEYS = {"metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
        "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"}
ROOFLINE_KEYS = {"bound", "achieved", "peak", "unit", "frac", "traffic"}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


@pytest.mark.parametrize("workload,lo,hi", [("c1", 1.0e9, 1.3e9), ("c4", 4.5e9, 5.8e9)])
def test_traffic_digest_is_read_from_the_profile(workload, lo, hi):
    sys.path.insert(0, ROOT)
    import bench
    d = bench.kernel_source_digest()
    assert len(d) == 16
    text = open(bench.PROFILE_SUMMARY[workload]).read()
    t = bench.measured_traffic(workload)
    if ("kernel_source_digest: " + d) in text and "hbm_bytes_per_launch" in text:
        assert t is not None and lo < t < hi
    else:
        assert t is None


@pytest.mark.gpu
def test_short_bench_prints_the_contract_line():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = subprocess.run([sys.executable, "bench.py", "--steps", "20", "--warmup", "4", "--pre-steps", "16", "--no-cpu", "--no-tts"],
                       cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    line = [l for l in r.stdout.splitlines() if l.startswith("{")][-1]
    out = json.loads(line)
    assert KEYS <= set(out) and ROOFLINE_KEYS <= set(out["roofline"])
    assert out["n_gpus"] == 1 and out["steps"] == 20 and out["value"] > 0
    assert out["roofline"]["bound"] == "hbm" and 0 < out["roofline"]["frac"] < 1
    assert out["config"]["workload"].startswith("plain single run, 4096x384x384")
    # a short run times every step's sweep
    assert out["roofline"]["timed_launches"] == 20 and out["roofline"]["sample_every"] == 1
