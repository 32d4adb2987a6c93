"""The benchmark's command-line contract: one JSON line with the fields the
measurement needs (GPU), and a clear refusal of more than one GPU (CPU)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert "one GPU" in (r.stdout + r.stderr)
    assert not [l for l in r.stdout.splitlines() if l.startswith("{")]


@pytest.mark.gpu
def test_bench_prints_one_json_line_with_roofline_and_cpu_baseline():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "20",
                        "--warmup", "5", "--no-extra"],
                       capture_output=True, text=True, timeout=280, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    rec = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in rec, k
    assert rec["n_gpus"] == 1 and rec["steps"] == 20 and rec["warmup"] == 5
    assert rec["value"] > 0 and rec["higher_is_better"] is True and rec["dtype"] == "f32"
    assert rec["config"]["workload"] == "taylor_green_4096x4096"
    roof = rec["roofline"]
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-3
    # achieved = 72 B per lattice update x nodes / time per step
    assert abs(roof["achieved"] - 72 * 4096 ** 2 / (rec["ms_per_step"] * 1e-3) / 1e9) \
        <= 1e-3 * roof["achieved"]
    # three time steps per launch: the launch lasts three steps' time, and
    # what HBM carries (when the committed counters match the source) stays
    # below the peak
    assert roof["updates_per_launch"] == 3 and roof["kernel"] == "sweep_tb3_kernel<f32>"
    assert rec["config"]["launch"]["steps_per_sweep"] == 3
    assert abs(roof["avg_duration_us"] - 3e3 * rec["ms_per_step"]) <= 2e-3 * roof["avg_duration_us"]
    if roof["traffic"] is not None:
        assert 0 < roof["traffic_frac"] < 1
    cpu = rec["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["cores"] >= 1 and cpu["value"] > 0
    assert cpu["unit"] == "MLUPS" and cpu["sample"]
    # the oracle on the two small configurations too, all cores and one thread
    assert set(cpu["configs"]) == {"taylor_green_64x64_x1000",
                                   "taylor_green_64x64_x1000_1thread",
                                   "double_shear_layer_1024x1024_x100",
                                   "double_shear_layer_1024x1024_x5_1thread"}
    assert all(c["MLUPS"] > 0 for c in cpu["configs"].values())
    # the timed configuration's accuracy against the oracle state of that sample
    acc = rec["accuracy"]
    assert acc["steps"] >= 1 and "oracle" in acc["reference"]
    assert 0 < acc["err_max"] <= 1e-5 and 0 < acc["err_L2"] <= 1e-5
    # the access-pattern ceiling beside the sweep's own figure
    pat = roof["access_pattern"]
    assert pat["kernel"].startswith("pattern_probe_kernel") and 0 < pat["frac"] < 1
    assert abs(pat["sweep_over_pattern"] - roof["achieved"] / pat["achieved"]) < 1e-3
