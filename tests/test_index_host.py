"""Host checks of the 32-bit index arithmetic of the binning.

The binary search that finds each bin's first point (index_math.h, used by the
sorted-input binning and the reproducible binning) is compiled for the host
and run at N_d = 2^30 (the largest accepted count) and 2^31 - 1 on a virtual
sorted key array; the C ABI rejects N_d above 2^30 before any device work.
"""
import ctypes
import os
import subprocess

import pytest

from paper_2409_08090_amd import mils

HERE = os.path.dirname(os.path.abspath(__file__))


def test_lower_bound_at_largest_counts(tmp_path):
    exe = tmp_path / "index_check"
    subprocess.run(["g++", "-O2", "-std=c++17", os.path.join(HERE, "index_check.cpp"), "-o",
                    str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")


@pytest.mark.parametrize("nd,ok", [(1, True), (2**30, True), (2**30 + 1, False), (2**31 - 1, False)])
def test_point_count_limit(nd, ok):
    lib = mils.load()
    p = mils.make_params(0.01, 0.01, 100)
    dummy = ctypes.c_void_p(16)  # never dereferenced: the check is host-only
    rc = lib.mils_check_periodogram_args(dummy, dummy, nd, ctypes.byref(p), dummy)
    assert (rc == 0) == ok, rc


@pytest.mark.parametrize("l0,l1,c", [(256, 256, 4), (512, 256, 2), (2048, 256, 8), (256, 2048, 4),
                                     (4096, 256, 4), (256, 8192, 8), (1024, 512, 2)])
def test_two_pass_fft_index_math(tmp_path, l0, l1, c):
    """The two-pass register-tile FFT's index arithmetic (fft2_index.h), run
    on the host: threads one after another, LDS exchanges bounds-checked and
    every read slot written in the same exchange; the result against the
    direct DFT at sampled modes (1e-12 relative)."""
    exe = tmp_path / "fft2_check"
    subprocess.run(["g++", "-O2", "-std=c++17", os.path.join(HERE, "fft2_check.cpp"), "-o",
                    str(exe)], check=True)
    r = subprocess.run([str(exe), str(l0), str(l1), str(c)], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
