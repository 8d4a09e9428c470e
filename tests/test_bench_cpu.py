"""The benchmark script's host logic (no GPU): the one-GPU guard, the
measured-traffic lookup that must refuse counters taken on other kernel
sources, and the figures of the vector-issue roof."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_only_for_the_current_kernel_sources(tmp_path):
    key = "stencil_tb_f64_T3_L512"
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps({key: {"bytes": 123, "source_sha256": bench.kernel_source_hash()}}))
    assert bench.traffic_for(str(path), key) == 123
    assert bench.traffic_for(str(path), "stencil_tb_f64_T2_L512") is None
    path.write_text(json.dumps({key: {"bytes": 123, "source_sha256": "0" * 64}}))
    assert bench.traffic_for(str(path), key) is None
    assert bench.traffic_for(str(tmp_path / "missing.json"), key) is None


def test_vector_issue_roof_figures():
    assert abs(bench.VALU_PEAK_TOPS - 39.3216) < 1e-9   # 256 x 4 x 16 lanes x 2.4 GHz
    assert bench.alu_ops_per_cell_update("f64", True) == 48
    assert bench.alu_ops_per_cell_update("f64", False) == 36
    assert bench.alu_ops_per_cell_update("f32", True) is None
