"""CPU oracle for the NUFFT Lomb-Scargle path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does, and this
package imports nothing from the product package.

The arithmetic lives in ``ls_oracle.c`` (plain C, OpenMP over frequencies): a
direct O(N_d) evaluation per frequency of the trigonometric sums of Eq. 1 /
Eq. 2 of the nifty-ls paper (Sec. 1), and the Lomb-Scargle periodogram as the
weighted least-squares fit of a sinusoid at each frequency.  This module only
compiles it and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ls_oracle.c")
_LIB = os.path.join(_HERE, "libls_oracle.so")

NORMALIZATIONS = {"standard": 0, "model": 1, "log": 2, "psd": 3}

_lib = None
_native = False


def _target(native: bool) -> str:
    return os.path.join(_HERE, "libls_oracle_native.so") if native else _LIB


def build(force: bool = True, native: bool = False) -> str:
    """Compile ls_oracle.c with gcc (no fast-math, no FP contraction).  The
    default build is -O2 for any x86-64 host; native=True builds -O3
    -march=native for the machine it runs on (the timed CPU baseline).
    Neither reassociates or contracts floating point, so both give the same
    values."""
    out = _target(native)
    if not force and os.path.exists(out):
        return out
    opt = ["-O3", "-march=native"] if native else ["-O2"]
    cmd = [
        "gcc", *opt, "-fPIC", "-shared", "-fopenmp", "-std=c11",
        "-fno-fast-math", "-ffp-contract=off", "-Wall",
        _SRC, "-o", out + ".tmp", "-lm",
    ]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def use_native() -> None:
    """Switch this process to the -O3 -march=native build (built here on
    first use)."""
    global _lib, _native
    if not _native:
        build(force=True, native=True)
        _native = True
        _lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = _target(_native)
    if not os.path.exists(path):
        build(native=_native)
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_trig_sums.argtypes = [dp, dp, ctypes.c_int64, ctypes.c_double,
                                     ctypes.c_double, ip, ctypes.c_int64, dp, dp]
    lib.oracle_trig_sums.restype = None
    lib.oracle_periodogram.argtypes = [dp, dp, dp, ctypes.c_int64, ctypes.c_double,
                                       ctypes.c_double, ip, ctypes.c_int64,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       dp, i32p]
    lib.oracle_periodogram.restype = ctypes.c_int
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _kidx(nf, k):
    if k is None:
        k = np.arange(nf, dtype=np.int64)
    return np.ascontiguousarray(k, dtype=np.int64)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def trig_sums(t, h, f0, df, nf=None, k=None):
    """sum_j h_j exp(+2 pi i (f0 + k df) t_j) for every requested k (complex128)."""
    lib = _load()
    t = _f64(t)
    h = _f64(h)
    assert t.shape == h.shape and t.ndim == 1
    k = _kidx(nf, k)
    re = np.empty(k.size)
    im = np.empty(k.size)
    lib.oracle_trig_sums(_dptr(t), _dptr(h), t.size, float(f0), float(df),
                         k.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), k.size,
                         _dptr(re), _dptr(im))
    return re + 1j * im


def periodogram(t, y, dy, f0, df, nf=None, k=None, normalization="standard",
                center_data=True, fit_mean=True, return_flags=False):
    """Lomb-Scargle power at f0 + k df (float64); see ls_oracle.c for the definition."""
    lib = _load()
    t = _f64(t)
    y = _f64(y)
    assert t.shape == y.shape and t.ndim == 1
    if dy is not None:
        dy = _f64(np.broadcast_to(dy, t.shape))
    k = _kidx(nf, k)
    p = np.empty(k.size)
    flags = np.empty(k.size, dtype=np.int32)
    rc = lib.oracle_periodogram(
        _dptr(t), _dptr(y), _dptr(dy) if dy is not None else None, t.size,
        float(f0), float(df), k.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), k.size,
        NORMALIZATIONS[normalization], int(bool(center_data)), int(bool(fit_mean)),
        _dptr(p), flags.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc != 0:
        raise ValueError(f"oracle_periodogram failed with code {rc} (constant data?)")
    return (p, flags) if return_flags else p
