"""The benchmark's command line, on the CPU: its defaults (the lattice
workload, the headline schedule among the modes, a bounded run) and its
refusal of more than one GPU before any GPU work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_defaults():
    sys.path.insert(0, ROOT)
    import bench
    a = bench.parse([])
    assert a.gpus == 1 and a.config == "cfg2"
    modes = a.modes.split(",")
    assert "f64" in modes and "bf16x3+L" in modes
    assert 1 <= a.steps <= 50 and 0 <= a.warmup <= 10
    assert a.pad in (32, 64)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""            # no JSON line
