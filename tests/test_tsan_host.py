"""The serving loop's threads under ThreadSanitizer (host only, no GPU):
tests/server_tsan_check.cpp replaces the HIP runtime and the library's
compute entry points with host stand-ins and drives server.cpp from several
client threads (submit, poll, wait, take), a warm-up and stats readers, then
a shutdown with requests in flight and injected lane failures.  Every result
is traced back to its request.  Built with ROCm's clang: the timed waits of
libstdc++ use pthread_cond_clockwait, which the ThreadSanitizer of the
system's g++ does not intercept (it then reports the waiting mutex as
double-locked)."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(not os.path.exists(CLANG), reason="needs ROCm's clang++")
def test_server_threads_under_tsan(tmp_path):
    exe = tmp_path / "server_tsan_check"
    cmd = [CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=thread", "-I/opt/rocm/include",
           "-D__HIP_PLATFORM_AMD__", os.path.join(HERE, "server_tsan_check.cpp"),
           os.path.join(ROOT, "paper_2409_08090_amd", "csrc", "server.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    env.pop("MILS_SERVER_FAIL_AFTER", None)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert r.stdout.strip().endswith("server ok")
