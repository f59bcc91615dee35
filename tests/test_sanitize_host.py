"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (g++, no
GPU): the planner over a sweep of sizes, tolerances, precisions and plan
kinds, and the plain host NUFFT on ragged single series, a batch and its FFT
(tests/sanitize_check.cpp).  Any finding aborts the program."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_planner_and_host_nufft_under_asan_ubsan(tmp_path):
    exe = tmp_path / "sanitize_check"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
           os.path.join(HERE, "sanitize_check.cpp"),
           os.path.join(ROOT, "paper_2409_08090_amd", "csrc", "plan.cpp"),
           os.path.join(ROOT, "hostnufft", "hostnufft.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert r.stdout.strip().endswith("plans ok")
