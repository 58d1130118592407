"""Host logic of bench.py (no GPU): the counter-summary lookup behind the
roofline's `traffic` field and the one-GPU guard."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _recorded(path):
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    return vals


@pytest.mark.parametrize("kernel", ["outer_lean_fwd", "outer_lean_bwd", "rows_lean"])
def test_traffic_is_read_only_for_the_recorded_sources(kernel):
    path = os.path.join(ROOT, "profiles", "%s_c5_3d_pmc.txt" % kernel)
    vals = _recorded(path)
    got = bench.read_traffic(kernel, "c5_3d", vals["kernel_src"])
    assert got == pytest.approx(float(vals["hbm_bytes_per_launch"]))
    assert bench.read_traffic(kernel, "c5_3d", "0" * 12) is None
    assert bench.read_traffic(kernel, "no_such_workload", vals["kernel_src"]) is None


def test_committed_counters_are_near_the_algorithmic_bytes():
    # forward outer pass of the 256^3 plan: 1.21 GB per launch by design
    vals = _recorded(os.path.join(ROOT, "profiles", "outer_lean_fwd_c5_3d_pmc.txt"))
    assert float(vals["hbm_bytes_per_launch"]) == pytest.approx(1207959552.0, rel=0.02)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr)
