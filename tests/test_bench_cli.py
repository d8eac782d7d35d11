"""The benchmark's command line without a GPU: more than one GPU is refused with a message, and the
workload list and defaults parse."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_defaults_parse():
    sys.path.insert(0, ROOT)
    import bench

    a = bench.parse([])
    assert a.gpus == 1 and a.workload == "capsule" and a.precision == "fp32"
    assert a.kin_relax == "jacobi" and a.max_inner == 100
