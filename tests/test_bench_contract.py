"""bench.py's contract pieces that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_work_counts():
    sys.path.insert(0, ROOT)
    import bench
    # p = 6: calL = 84; symmetric Gram 84*85 + rhs 2*84 + basis 84
    assert bench.gram_flops_per_point(84) == 84 * 85 + 3 * 84
    assert bench.eval_flops_per_query(84) == 2 * 84
    # p = 6: 455 power moments + 84 weighted + 1, 91 + 28 runs, 36 powers
    assert bench.moment_flops_per_point(6) == 2 * (455 + 84 + 1) + 119 + 36
    assert bench.bmoment_flops_per_point(6) == 2 * 84 + 28 + 18
    assert bench.base_moment_flops_per_point(6) == 2 * 455 + 91 + 36
    assert bench.solve_flops_per_node(84) == 84 ** 3 / 3 + 2 * 84 * 84


def test_refit_rooflines_from_launch_records():
    sys.path.insert(0, ROOT)
    import bench
    # two steps; the refit's factor class covered 100 nodes in 2 ms in total
    kern = {"refit_factor": dict(launches=10, ms_per_step=1.0, avg_launch_ms=0.2, units=100.0),
            "refit_residual": dict(launches=10, ms_per_step=0.5, avg_launch_ms=0.1, units=2.0e6)}
    r = bench.refit_rooflines(kern, 6, 84, 4, 2)
    assert abs(r["refit_factor"]["achieved"] - 100 * 84 ** 3 / 3 / 2e-3 / 1e12) < 1e-12
    assert r["refit_factor"]["unit"] == "TFLOP/s" and r["refit_factor"]["peak"] == 78.6
    assert abs(r["refit_residual"]["achieved"] - 2e6 * (16 + 12) / 1e-3 / 1e9) < 1e-9
    r8 = bench.refit_rooflines(kern, 6, 84, 4, 2, 8)
    assert abs(r8["refit_residual"]["achieved"] - 2e6 * (16 + 1.5) / 1e-3 / 1e9) < 1e-9
    assert r["refit_residual"]["bound"] == "hbm"
