"""Host-side logic of bench.py (no GPU): the one-GPU guard, the lookup of the
committed counter summary and the CPU description of the baseline."""
import os
import re
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_kernel_source_hash_and_traffic_lookup():
    h = bench.kernel_sources_sha256()
    assert re.fullmatch(r"[0-9a-f]{64}", h)
    for which in ("pre", "post"):
        t = bench.measured_traffic("c2_spheres_256", which)
        # a number only while the committed summary was taken from these sources
        assert t is None or t > 0
    assert bench.measured_traffic("no_such_workload", "post") is None


def test_host_cpu_description():
    d = bench.host_cpu()
    assert d["usable_cores"] >= 1
    assert d["cpu_model"] is None or isinstance(d["cpu_model"], str)
