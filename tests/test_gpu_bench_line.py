"""bench.py's output line: a short run on the smallest workload settings,
parsed and checked for the fields the measurement is reported with (metric,
value, unit, steps, the roofline object of the dominant kernel, the oracle's
CPU baseline) and for the parity flags it computes along the way."""
import json
import os
import subprocess
import sys

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_prints_one_complete_json_line():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "5", "--warmup", "1", "--bbox-steps", "5",
           "--map-reps", "1", "--cpu-seconds", "0.1", "--no-cpu-one-thread", "--repeats", "2",
           "--batch-steps", "3", "--batch-seq-steps", "1", "--serve-seconds", "0", "--large-steps", "3",
           "--packed"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 5 and d["warmup"] == 1 and d["dtype"] == "u8"
    assert d["value"] > 0 and d["unit"] == "cell-updates/s" and d["config"]["workload"] == "triangle_r16"
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["peak"] == 8000.0 and rf["unit"] == "GB/s"
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-9 and rf["achieved"] > 0
    assert rf["alg_bytes_per_launch"] == 2 * 3 ** 16
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and cb["sample"]
    # the checks the run makes on the way
    assert d["compact_equals_bbox"] is True
    assert d["maps"]["nu_of_lambda_is_identity"] is True
    assert d["packed_state"]["equals_byte_step"] is True
    assert d["batch"]["matches_sequential"] is True and d["batch"]["small_instances"]["same"] is True
    assert d["small_triangle_r10"]["graph_equals_eager"] is True
    assert d["compact_repeats"]["steps_each"] >= 100
    for nm in ("carpet_r9", "hfractal_r10"):
        lw = d["large_workloads"][nm]
        assert lw["compact_equals_bbox"] is True and lw["steps"] == 3
        assert abs(lw["roofline_frac"] - lw["alg_gbps"] / 8000.0) < 1e-9
        assert "traffic_over_alg" in lw and "bbox_traffic_over_alg" in lw


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr)
