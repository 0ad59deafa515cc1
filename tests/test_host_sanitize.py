"""The host code of the symbolic plan (step 1 of Fig. 2) under
AddressSanitizer and UndefinedBehaviorSanitizer: plan.cpp and a driver
(tests/native/plan_sanitize.cpp) built with g++ for the CPU, run on a
water-like pattern, generated chains of ragged block sizes and every
malformed pattern the plan must refuse.  No device code is built or run."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _write_pattern(m, path):
    with open(path, "wb") as f:
        f.write(np.int32(m.n_atoms).tobytes())
        f.write(np.int64(m.row_idx.shape[0]).tobytes())
        f.write(np.ascontiguousarray(m.block_size, np.int32).tobytes())
        f.write(np.ascontiguousarray(m.col_ptr, np.int64).tobytes())
        f.write(np.ascontiguousarray(m.row_idx, np.int32).tobytes())
        f.write(np.ascontiguousarray(m.panel_off, np.int64).tobytes())


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(os.path.join(ROCM, "include", "hip")),
                    reason="needs g++ and the HIP headers")
def test_plan_under_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_sanitize")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "native", "plan_sanitize.cpp"),
           os.path.join(ROOT, "paper_2205_14741_amd", "csrc", "plan.cpp"),
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    pat = str(tmp_path / "water.bin")
    _write_pattern(synth.water_system(12, 1.6, 4), pat)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe, pat], capture_output=True, text=True, env=env, timeout=120)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "plan checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
