"""The benchmark's command line, on the CPU: its defaults (the water-like
workload, the float64 reference and the headline schedule, a bounded run)
and its refusal of more than one GPU before any GPU work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_defaults():
    sys.path.insert(0, ROOT)
    import bench
    a = bench.parse([])
    assert a.gpus == 1 and a.config == "cfg3" and a.modes is None
    assert 1 <= a.steps <= 50 and 0 <= a.warmup <= 10 and a.ref_steps >= 1
    assert a.pad in (32, 64)
    a = bench.parse(["--steps", "20", "--warmup", "5", "--config", "cfg4"])
    assert (a.steps, a.warmup, a.config) == (20, 5, "cfg4")
    assert "cfg3" in bench.WORKLOADS and "cfg4" in bench.WORKLOADS
    assert a.fermi == 0.0     # the sign path unless a finite temperature is asked for
    a = bench.parse(["--fermi", "20", "--config", "cfg2"])
    assert a.fermi == 20.0 and a.config == "cfg2"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""            # no JSON line
