"""Host-side behaviour of bench.py that needs no GPU: a run on more than one
GPU is refused with a message (one GPU only; the sharding is a design note),
and the description of the host the oracle runs on is plain host code."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert '"metric"' not in r.stdout


def test_host_cpu_description():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.host_cpu()
    assert set(h) == {"model", "logical_cpus", "usable_cpus"}
    assert h["logical_cpus"] is None or h["logical_cpus"] >= 1
