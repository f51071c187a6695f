"""Host-side logic of bench.py (no GPU): the algorithmic operation counts behind the
roofline, the roofline entry's arithmetic against the published FP64 peak, the lookup of
the measured HBM traffic (only for the sources and tile shape it was taken with), and the
refusal of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_operation_counts():
    # one WENO-theta reconstruction and one characteristic interface of the 2D Euler system
    assert bench.WENO_OPS == 132
    assert bench.euler_interface_ops(2) == 1555
    assert bench.euler_interface_ops(1) < bench.euler_interface_ops(2) < bench.euler_interface_ops(3)
    # one x sweep of 4096^2: 4096 lines of 4097 interfaces and 4096^2 cells
    n = (4096, 4096)
    ops = bench.sweep_ops(2, n, 0, False)
    assert ops == 4096 * 4097 * 1555 + 4096 * 4096 * bench.euler_cell_ops(2, False)
    final = bench.sweep_ops(2, n, 1, True)
    assert final - ops == 4096 * 4096 * (bench.euler_cell_ops(2, True) - bench.euler_cell_ops(2, False))
    # the fused 2D stage is credited with both directions' work
    case = type("C", (), {"ndim": 2, "n": n})()
    assert bench.kernel_ops(case, "stage_2d", True) == (bench.sweep_ops(2, n, 0, False) +
                                                        bench.sweep_ops(2, n, 1, True))


def test_roofline_entry_against_the_published_peak():
    e = bench.roofline_entry("sweep_y_final", 2.7e10, tot_ms=90.0, launches=100, traffic=2.0e9)
    achieved = 2.7e10 / 0.9e-3
    assert e["bound"] == "alu" and e["unit"] == "TFLOP/s"
    assert e["peak"] == pytest.approx(78.6)
    assert e["achieved"] == pytest.approx(achieved / 1e12)
    assert e["frac"] == pytest.approx(achieved / 78.6e12)
    assert e["frac_of_lane_issue_rate"] == pytest.approx(achieved / (256 * 64 * 2.4e9))
    assert e["traffic"] == 2.0e9 and e["avg_launch_ms"] == pytest.approx(0.9)


def test_measured_traffic_only_for_its_sources_and_tile():
    path = os.path.join(ROOT, "profiles", "traffic_euler2d_4096_fp64_fast.txt")
    if not os.path.exists(path):
        pytest.skip("no traffic summary committed")
    kv = dict(line.split("=", 1) for line in open(path) if "=" in line and not line.startswith("#"))
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    got = bench.measured_traffic("sweep_x", kv["y_tile"], "fp64_fast")
    if kv["sources_sha256"] == bench.kernel_sources_hash():
        assert got == float(kv["sweep_x.bytes"])
        assert bench.measured_traffic("sweep_y_final", "16x15", "fp64_fast") is None
    else:
        assert got is None
    assert bench.measured_traffic("sweep_x", kv["y_tile"], "no_such_precision") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""                 # no JSON line for a refused run
