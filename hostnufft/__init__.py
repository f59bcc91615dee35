"""Plain host FP64 NUFFT Lomb-Scargle periodogram -- a CPU BASELINE for timing.

``hostnufft.cpp`` (C++, OpenMP) evaluates the same periodogram as the GPU
library with the same method (type-1 NUFFT of the paper's Sec. 1: spread with
the exponential-of-semicircle kernel, FFT, deconvolution; then the
least-squares power), with its own host FFT, on every host core.  It stands in
for the CPU backend the paper times (Sec. 2, Sec. 2.1).  The GPU library never
imports or calls it; ``bench.py`` times it beside the GPU path and the tests
pin it against the oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hostnufft.cpp")

NORMALIZATIONS = {"standard": 0, "model": 1, "log": 2, "psd": 3}
_libs: dict = {}


def lib_path(native: bool = False) -> str:
    return os.path.join(_HERE, "libhostnufft_native.so" if native else "libhostnufft.so")


def build(native: bool = False) -> str:
    """Compile hostnufft.cpp with g++ (-O3, OpenMP; -march=native for the
    machine it runs on when native, otherwise portable x86-64)."""
    out = lib_path(native)
    arch = ["-march=native"] if native else []
    cmd = ["g++", "-O3", *arch, "-fPIC", "-shared", "-fopenmp", "-std=c++17",
           "-fno-fast-math", "-Wall", _SRC, "-o", out + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _load(native: bool = False):
    if native in _libs:
        return _libs[native]
    path = lib_path(native)
    if not os.path.exists(path):
        build(native)
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.hostnufft_num_threads.restype = ctypes.c_int
    lib.hostnufft_plan.argtypes = [ctypes.c_int64, ctypes.c_double]
    lib.hostnufft_plan.restype = ctypes.c_int64
    lib.hostnufft_periodogram.argtypes = [dp, dp, dp, ctypes.c_int64, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_int64, ctypes.c_double,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, dp]
    lib.hostnufft_periodogram.restype = ctypes.c_int
    lib.hostnufft_batch.argtypes = [ctypes.c_int64, ip, dp, dp, dp, ip, dp, dp, ctypes.c_double,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp,
                                    i32p]
    lib.hostnufft_batch.restype = ctypes.c_int
    lib.hostnufft_fft.argtypes = [dp, ctypes.c_int64, ctypes.c_int]
    lib.hostnufft_fft.restype = ctypes.c_int
    _libs[native] = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_threads() -> int:
    return len(os.sched_getaffinity(0))


def plan(nf: int, eps: float = 1e-9, native: bool = False) -> int:
    """Build (and cache) the plan for nf frequencies; returns its grid size."""
    return int(_load(native).hostnufft_plan(int(nf), float(eps)))


def periodogram(t, y, dy, f0, df, nf, eps=1e-9, normalization="standard", center_data=True,
                fit_mean=True, threads=None, native=False):
    """Power at f0 + k df, k < nf (float64 numpy array)."""
    lib = _load(native)
    t, y = _f64(t), _f64(y)
    dyv = None if dy is None else _f64(np.broadcast_to(dy, t.shape))
    out = np.empty(int(nf))
    rc = lib.hostnufft_periodogram(_dp(t), _dp(y), _dp(dyv) if dyv is not None else None,
                                   t.size, float(f0), float(df), int(nf), float(eps),
                                   NORMALIZATIONS[normalization], int(bool(center_data)),
                                   int(bool(fit_mean)), int(threads or default_threads()),
                                   _dp(out))
    if rc != 0:
        raise ValueError(f"hostnufft_periodogram failed with code {rc}")
    return out


def batch(curves, eps=1e-9, threads=None, native=False):
    """Periodograms of many series (objects with t, y, dy, f0, df, nf); returns
    the concatenated powers and the per-series status codes."""
    lib = _load(native)
    nd_off = np.zeros(len(curves) + 1, np.int64)
    nf_off = np.zeros(len(curves) + 1, np.int64)
    nd_off[1:] = np.cumsum([c.t.size for c in curves])
    nf_off[1:] = np.cumsum([c.nf for c in curves])
    t = _f64(np.concatenate([c.t for c in curves]))
    y = _f64(np.concatenate([c.y for c in curves]))
    dy = _f64(np.concatenate([np.broadcast_to(c.dy, c.t.shape) for c in curves]))
    f0 = _f64([c.f0 for c in curves])
    df = _f64([c.df for c in curves])
    out = np.empty(int(nf_off[-1]))
    st = np.zeros(len(curves), np.int32)
    ipp = ctypes.POINTER(ctypes.c_int64)
    lib.hostnufft_batch(len(curves), nd_off.ctypes.data_as(ipp), _dp(t), _dp(y), _dp(dy),
                        nf_off.ctypes.data_as(ipp), _dp(f0), _dp(df), float(eps), 0, 1, 1,
                        int(threads or default_threads()), _dp(out),
                        st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return out, st


def fft(x, threads=None):
    """The host FFT alone: X[m] = sum_l x[l] exp(+2 pi i l m / n)."""
    lib = _load(False)
    a = np.ascontiguousarray(np.asarray(x, dtype=np.complex128)).copy()
    v = a.view(np.float64)
    lib.hostnufft_fft(_dp(v), a.size, int(threads or default_threads()))
    return a
