"""The benchmark script's host logic (no GPU): the one-GPU guard, the
measured-traffic lookup that must refuse counters taken on other kernel
sources, instantiations, grids or z-chunks, and the roofline figures."""
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


def test_traffic_only_for_the_current_kernel_and_launch(tmp_path):
    cfg = dict(tile=6, tblock=3, zchunk=128, tx=64, ty=22)
    kname = bench.kernel_name(cfg, "f64", True)
    assert kname == "stencil_tb<double, 16, 22, 3, 512, true>"
    key = bench.traffic_key(kname, 512, 128)
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps({key: {"bytes": 123, "source_sha256": bench.kernel_source_hash()}}))
    assert bench.traffic_for(str(path), key) == 123
    assert bench.traffic_for(str(path), bench.traffic_key(kname, 512, 64)) is None     # other z-chunk
    assert bench.traffic_for(str(path), bench.traffic_key(kname, 1024, 128)) is None   # other grid
    other = bench.kernel_name(dict(cfg, tblock=2, ty=24), "f64", True)
    assert bench.traffic_for(str(path), bench.traffic_key(other, 512, 128)) is None    # other instantiation
    path.write_text(json.dumps({key: {"bytes": 123, "source_sha256": "0" * 64}}))
    assert bench.traffic_for(str(path), key) is None                                   # other sources
    assert bench.traffic_for(str(tmp_path / "missing.json"), key) is None
    assert any("gs_api.cpp" in f for f in bench.KERNEL_SOURCES)
    assert any("gs_launch.hpp" in f for f in bench.KERNEL_SOURCES)


def test_kernel_sources_closed_under_local_includes():
    """Every library header a hashed source includes is hashed too, so a
    change to it also invalidates the stored counter bytes."""
    import os
    import re
    hashed = set(bench.KERNEL_SOURCES)
    for f in bench.KERNEL_SOURCES:
        d = os.path.dirname(f)
        with open(os.path.join(bench.ROOT, f)) as fh:
            for inc in re.findall(r'#include "([^"]+)"', fh.read()):
                path = os.path.normpath(os.path.join(d, inc))
                if path.startswith("paper_2309_10292_amd/csrc/"):
                    assert path in hashed, (f, inc)


def test_roofline_fraction_is_of_the_binding_roof():
    assert abs(bench.VALU_PEAK_TOPS - 39.3216) < 1e-9   # 256 x 4 x 16 lanes x 2.4 GHz
    assert bench.alu_ops_per_cell_update("f64", True) == 48
    assert bench.alu_ops_per_cell_update("f64", False) == 35
    assert bench.alu_ops_per_cell_update("f32", True) is None
    cells = 512 ** 3
    # a T = 3 launch of 1.3 ms: one pass of 32 B per cell is 4.29e9 B
    r = bench.roofline("f64", True, cells, 3, 1.3, None)
    assert r["hbm"]["bytes_per_launch"] == 32 * cells
    assert abs(r["hbm"]["achieved"] - 32 * cells / 1.3e-3 / 1e9) < 0.1
    assert abs(r["alu"]["achieved"] - 48 * 3 * cells / 1.3e-3 / 1e12) < 0.01
    assert r["frac"] == max(r["hbm"]["frac"], r["alu"]["frac"]) <= 1.0
    assert r["bound"] == ("alu" if r["alu"]["frac"] > r["hbm"]["frac"] else "hbm")
    # the Eq. 5a-style figure counts every fused step and may exceed the peak
    assert abs(r["effective"]["gbs"] - 3 * 32 * cells / 1.3e-3 / 1e9) < 0.1
    # a launch at the binding roof's time gives frac 1
    t_roof = max(32 * cells / 8e12, 48 * 3 * cells / (bench.VALU_PEAK_TOPS * 1e12)) * 1e3
    assert abs(bench.roofline("f64", True, cells, 3, t_roof, None)["frac"] - 1.0) < 1e-3
    m = bench.roofline("f64", True, cells, 3, 1.3, 4.7e9)["measured"]
    assert abs(m["ratio_to_one_pass"] - 4.7e9 / (32 * cells)) < 1e-3
