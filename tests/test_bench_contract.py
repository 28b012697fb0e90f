"""The benchmark's command-line contract: one GPU only (a request for more
exits with a message, before any device work), and on a GPU one JSON line
with the fields the headline measurement promises."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


@pytest.mark.gpu
def test_headline_json_line():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "5",
                        "--warmup", "2", "--no-cpu-baseline"],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    line = json.loads(r.stdout.strip().splitlines()[-1])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                "roofline"):
        assert key in line, key
    assert line["n_gpus"] == 1 and line["steps"] == 5 and line["value"] > 0
    assert line["config"]["workload"] == "acoustic2d_2048_fd4_order8_k6"
    roof = line["roofline"]
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-9
    # the metric's second half: forward + adjoint at fixed error vs plain,
    # with the adjoint pass kernel's own roofline
    fa = line["fwd_adj"]
    assert fa["unit"] == "s" and fa["value"] > 0
    assert fa["speedup_vs_plain"]["fp64"] > 1.0
    assert fa["fp32_stepping"]["grad_c2_rel_err_vs_fp64"] < 1e-3
    ar = fa["roofline"]
    assert ar["kernel"].startswith("gbs::adj_pass2d<double") and ar["launches"] > 0
    assert abs(ar["frac"] - ar["achieved"] / ar["peak"]) < 1e-9
    # the batch workload in both precisions, faster than the plain FP64 form,
    # FP32 within its stated error
    bt = line["batch64"]
    assert bt["f64"]["speedup_vs_plain_fp64"] > 1.0 and bt["f64"]["steps"] == 100
    assert bt["f32"]["ms_per_step"] < bt["f64"]["ms_per_step"]
    assert bt["f32"]["max_rel_err_vs_fp64"] < 1e-4
    for dt in ("f64", "f32"):
        bw = bt[dt]["bandwidth"]
        assert 0.0 < bw["frac"] < 1.0 and abs(bw["frac"] - bw["achieved"] / bw["peak"]) < 1e-9
    assert bt["f32"]["bandwidth"]["method_bytes_per_step"] < bt["f64"]["bandwidth"]["method_bytes_per_step"]
    # the 3-D forward with 8 right-hand sides
    a3 = line["acoustic3d"]
    assert a3["config"]["grid"] == [384, 384, 384] and a3["config"]["n_rhs"] == 8
    assert a3["speedup_vs_plain"]["fp64"] > 1.0 and a3["speedup_vs_plain"]["fp32"] > 1.0
    assert a3["fp32_max_rel_err_vs_fp64_pressure"] < 1e-4
