"""Thin ctypes binding of libmils (include/mils.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libmils.so.  torch is used for device memory and streams; arrays
are passed to the library as raw device pointers.  There is no CPU fallback:
if libmils.so is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import math
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build, unless MILS_LIB names another build of the same library
LIB_PATH = os.environ.get("MILS_LIB") or os.path.join(HERE, "libmils.so")

MILS_OK = 0
MILS_ERR_INVALID_ARG = -1
MILS_ERR_DEGENERATE = -2
MILS_ERR_OOM = -3
MILS_ERR_DEVICE = -4
MILS_ERR_UNSUPPORTED = -5
MILS_ERR_BUSY = -6
MILS_ERR_CANCELLED = -7
MILS_ERR_TIMEOUT = -8

PRECISIONS = {"fp64": 0, "fp32": 1}
NORMALIZATIONS = {"standard": 0, "model": 1, "log": 2, "psd": 3}
MILS_CENTER_DATA = 1
MILS_FIT_MEAN = 2
MILS_DETERMINISTIC = 4


class mils_params(ctypes.Structure):
    _fields_ = [("f0", ctypes.c_double), ("df", ctypes.c_double), ("nf", ctypes.c_int64),
                ("eps", ctypes.c_double), ("precision", ctypes.c_int32),
                ("normalization", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class mils_plan_desc(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("width", ctypes.c_int32), ("beta", ctypes.c_double),
                ("n", ctypes.c_int64), ("npass", ctypes.c_int32), ("len", ctypes.c_int32 * 4),
                ("tile", ctypes.c_int32), ("bin", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_uint64), ("last_rows", ctypes.c_int32),
                ("last_lds_bytes", ctypes.c_int32), ("first_cols", ctypes.c_int32),
                ("first_lds_bytes", ctypes.c_int32), ("big", ctypes.c_int32),
                ("fft2", ctypes.c_int32)]


class mils_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("lanes", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("queue_capacity", ctypes.c_int32),
                ("tick_us", ctypes.c_int32)]


class mils_request(ctypes.Structure):
    _fields_ = [("t", ctypes.c_void_p), ("y", ctypes.c_void_p), ("dy", ctypes.c_void_p),
                ("nd", ctypes.c_int64), ("params", mils_params)]


class mils_request_stats(ctypes.Structure):
    _fields_ = [("submit_s", ctypes.c_double), ("start_s", ctypes.c_double),
                ("done_s", ctypes.c_double), ("status", ctypes.c_int32),
                ("batch_size", ctypes.c_int32)]


class mils_server_counters(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("inflight_bytes", ctypes.c_uint64), ("peak_inflight_bytes", ctypes.c_uint64),
                ("latency_p50_ms", ctypes.c_double), ("latency_p99_ms", ctypes.c_double),
                ("latency_max_ms", ctypes.c_double), ("sums_per_s", ctypes.c_double),
                ("mean_batch", ctypes.c_double), ("failed", ctypes.c_uint64),
                ("dead_lanes", ctypes.c_uint64), ("plans_built", ctypes.c_uint64),
                ("plan_build_ms", ctypes.c_double)]


class MilsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"libmils error {status}: {message}")
        self.status = status


_lib = None
_lock = threading.Lock()

# Exported symbols and their ctypes signatures (mirrors include/mils.h).
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I64P = ctypes.POINTER(ctypes.c_int64)
SIGNATURES = {
    "mils_version": ([], ctypes.c_int),
    "mils_status_str": ([ctypes.c_int], ctypes.c_char_p),
    "mils_last_error": ([_P], ctypes.c_char_p),
    "mils_context_create": ([ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(_P)], ctypes.c_int),
    "mils_context_destroy": ([_P], ctypes.c_int),
    "mils_context_set_graphs": ([_P, ctypes.c_int], ctypes.c_int),
    "mils_context_set_fft2": ([_P, ctypes.c_int], ctypes.c_int),
    "mils_plan_info": ([_P, ctypes.c_int64, ctypes.POINTER(mils_params),
                        ctypes.POINTER(mils_plan_desc)], ctypes.c_int),
    "mils_batch_tuning": ([_P, ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)],
                          ctypes.c_int),
    "mils_kernel_transform": ([_P, ctypes.POINTER(mils_params), ctypes.c_int64, _P, _P,
                               ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "mils_kernel_table": ([_P, ctypes.POINTER(mils_params), _P, ctypes.POINTER(ctypes.c_int32),
                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                           ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "mils_check_periodogram_args": ([_P, _P, ctypes.c_int64, ctypes.POINTER(mils_params), _P],
                                    ctypes.c_int),
    "mils_trig_sums": ([_P, _P, _P, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                        ctypes.c_int64, ctypes.c_double, ctypes.c_int32, _P, _P], ctypes.c_int),
    "mils_periodogram": ([_P, _P, _P, _P, ctypes.c_int64, ctypes.POINTER(mils_params), _P, _P],
                         ctypes.c_int),
    "mils_periodogram_async": ([_P, _P, _P, _P, ctypes.c_int64, ctypes.POINTER(mils_params),
                                _P, _P], ctypes.c_int),
    "mils_periodogram_noalloc": ([_P, _P, _P, _P, ctypes.c_int64, ctypes.POINTER(mils_params),
                                  _P, _P], ctypes.c_int),
    "mils_context_status": ([_P], ctypes.c_int),
    "mils_context_illposed": ([_P], ctypes.c_int64),
    "mils_periodogram_batch": ([_P, ctypes.c_int64, _I64P, _P, _P, _P, _I64P, _D, _D,
                                ctypes.POINTER(mils_params), _P,
                                ctypes.POINTER(ctypes.c_int32), _P], ctypes.c_int),
    "mils_direct_periodogram": ([_P, _P, _P, _P, ctypes.c_int64, ctypes.POINTER(mils_params),
                                 _P, _P], ctypes.c_int),
    "mils_direct_trig_sums": ([_P, _P, _P, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                               ctypes.c_int64, _P, _P], ctypes.c_int),
    "mils_periodogram_shared_t": ([_P, _P, _P, _P, ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_int64, ctypes.POINTER(mils_params), _P,
                                   ctypes.POINTER(ctypes.c_int32), _P], ctypes.c_int),
    "mils_profile_enable": ([_P, ctypes.c_int], ctypes.c_int),
    "mils_profile_stage_name": ([ctypes.c_int], ctypes.c_char_p),
    "mils_profile_stages": ([_P, ctypes.c_uint32], ctypes.c_int),
    "mils_profile_read": ([_P, _D, _I64P], ctypes.c_int),
    "mils_server_create": ([ctypes.c_int, ctypes.POINTER(mils_server_config), ctypes.POINTER(_P)],
                           ctypes.c_int),
    "mils_server_submit": ([_P, ctypes.POINTER(mils_request), ctypes.POINTER(ctypes.c_uint64)],
                           ctypes.c_int),
    "mils_server_poll": ([_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "mils_server_wait": ([_P, ctypes.c_uint64, ctypes.c_int64], ctypes.c_int),
    "mils_server_take": ([_P, ctypes.c_uint64, _P, ctypes.POINTER(mils_request_stats)],
                         ctypes.c_int),
    "mils_server_stats": ([_P, ctypes.POINTER(mils_server_counters)], ctypes.c_int),
    "mils_context_set_batch_onchip": ([_P, ctypes.c_int], ctypes.c_int),
    "mils_context_batch_onchip": ([_P], ctypes.c_int64),
    "mils_server_warm": ([_P, ctypes.POINTER(mils_params), ctypes.c_int64], ctypes.c_int),
    "mils_server_last_error": ([_P], ctypes.c_char_p),
    "mils_server_destroy": ([_P], ctypes.c_int),
}

MILS_NUM_STAGES = 11


def load():
    """Load libmils.so (raises when it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2409_08090_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
        return lib


def status_str(code: int) -> str:
    return load().mils_status_str(code).decode()


def version() -> int:
    return int(load().mils_version())


class Context:
    """A libmils context on one device (device=-1: host-only planning context)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        lib = load()
        h = _P()
        rc = lib.mils_context_create(int(device), int(hbm_budget_bytes), ctypes.byref(h))
        if rc != MILS_OK:
            raise MilsError(rc, lib.mils_last_error(None).decode())
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            load().mils_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return load().mils_last_error(self.handle).decode()

    def set_fft2(self, enable: bool):
        """Allow (or not) the two-pass register-tile FFT for this context's
        single-series calls."""
        self.check(load().mils_context_set_fft2(self.handle, int(bool(enable))))

    def set_batch_onchip(self, enable: bool):
        """Batched series whose grids fit LDS run whole in one workgroup."""
        self.check(load().mils_context_set_batch_onchip(self.handle, int(bool(enable))))

    def batch_onchip(self) -> int:
        """Series of the last batch built on this context that ran on chip."""
        return int(load().mils_context_batch_onchip(self.handle))

    def set_graphs(self, enable: bool):
        """Graph replay of repeated single-series calls (on by default)."""
        self.check(load().mils_context_set_graphs(self.handle, int(bool(enable))))

    def profile_enable(self, enable: bool = True, stages=None):
        """Per-stage HIP-event timing; stages: names to time (None: all)."""
        lib = load()
        mask = 0xFFFFFFFF
        if stages is not None:
            names = [lib.mils_profile_stage_name(i).decode() for i in range(MILS_NUM_STAGES)]
            mask = sum(1 << names.index(n) for n in stages)
        self.check(lib.mils_profile_stages(self.handle, mask))
        self.check(lib.mils_profile_enable(self.handle, int(bool(enable))))

    def profile_read(self) -> dict:
        """{stage name: (total ms, launches)} since the last read / enable."""
        import numpy as np
        ms = np.zeros(MILS_NUM_STAGES)
        n = np.zeros(MILS_NUM_STAGES, dtype=np.int64)
        self.check(load().mils_profile_read(self.handle, ms.ctypes.data_as(_D),
                                            n.ctypes.data_as(_I64P)))
        lib = load()
        return {lib.mils_profile_stage_name(i).decode(): (float(ms[i]), int(n[i]))
                for i in range(MILS_NUM_STAGES) if n[i]}

    def batch_tuning(self, nf: int, eps: float, precision: str = "fp64"):
        """(sigma, tile_max) the batch autotuner chose for series of nf
        frequencies (sigma 0.0: the planner's choice), or None if undecided."""
        sg = ctypes.c_double()
        tm = ctypes.c_int32()
        rc = load().mils_batch_tuning(self.handle, int(nf), float(eps), PRECISIONS[precision],
                                      ctypes.byref(sg), ctypes.byref(tm))
        return (sg.value, tm.value) if rc == MILS_OK else None

    def check(self, rc: int):
        if rc != MILS_OK:
            raise MilsError(rc, self.last_error())
        return rc


_contexts: dict[int, Context] = {}


def default_context(device: int | None = None) -> Context:
    import torch
    if device is None:
        device = torch.cuda.current_device()
    with _lock:
        ctx = _contexts.get(device)
    if ctx is None:
        ctx = Context(device)
        with _lock:
            _contexts[device] = ctx
    return ctx


def make_params(f0, df, nf, eps=1e-9, precision="fp64", normalization="standard",
                center_data=True, fit_mean=True, deterministic=False) -> mils_params:
    flags = ((MILS_CENTER_DATA if center_data else 0) | (MILS_FIT_MEAN if fit_mean else 0) |
             (MILS_DETERMINISTIC if deterministic else 0))
    return mils_params(float(f0), float(df), int(nf), float(eps), PRECISIONS[precision],
                       NORMALIZATIONS[normalization], flags)


def kernel_table(nf, eps=1e-9, precision="fp64", f0=0.01, df=0.01):
    """(coef[ncoef, kmax], width, beta) of the spreading-kernel polynomials of a
    plan (host only, no GPU needed)."""
    import numpy as np
    lib = load()
    ctx = Context(-1)
    p = make_params(f0, df, nf, eps, precision)
    buf = np.zeros(64 * 64, dtype=np.float64)
    nc, km, wd, be = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    ctx.check(lib.mils_kernel_table(ctx.handle, ctypes.byref(p), buf.ctypes.data, ctypes.byref(nc),
                                    ctypes.byref(km), ctypes.byref(wd), ctypes.byref(be)))
    ctx.close()
    return buf[: nc.value * km.value].reshape(nc.value, km.value).copy(), wd.value, be.value


def kernel_transform(nf, modes, eps=1e-9, precision="fp64"):
    """(1 / phihat(m) for each mode m, grid size n) of the plan of nf
    frequencies (host only, no GPU needed)."""
    import numpy as np
    lib = load()
    ctx = Context(-1)
    p = make_params(0.01, 0.01, nf, eps, precision)
    m = np.ascontiguousarray(modes, dtype=np.int64)
    out = np.empty(m.size)
    n = ctypes.c_int64()
    try:
        ctx.check(lib.mils_kernel_transform(ctx.handle, ctypes.byref(p), m.size, m.ctypes.data,
                                            out.ctypes.data, ctypes.byref(n)))
    finally:
        ctx.close()
    return out, int(n.value)


def plan_info(nd, nf, eps=1e-9, precision="fp64", f0=0.01, df=0.01) -> dict:
    """Planner decision for a periodogram (host only, no GPU needed)."""
    lib = load()
    ctx = Context(-1)
    p = make_params(f0, df, nf, eps, precision)
    d = mils_plan_desc()
    ctx.check(lib.mils_plan_info(ctx.handle, int(nd), ctypes.byref(p), ctypes.byref(d)))
    out = {"sigma": d.sigma, "width": d.width, "beta": d.beta, "n": d.n, "npass": d.npass,
           "len": list(d.len)[:d.npass], "tile": d.tile, "bin": d.bin,
           "workspace_bytes": d.workspace_bytes, "last_rows": d.last_rows,
           "last_lds_bytes": d.last_lds_bytes, "first_cols": d.first_cols,
           "first_lds_bytes": d.first_lds_bytes, "big": d.big, "fft2": d.fft2}
    ctx.close()
    return out


def _dev_f64(x, name):
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP torch tensor")
    if x.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return x


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def periodogram(t, y, dy, f0, df, nf, eps=1e-9, precision="fp64", normalization="standard",
                center_data=True, fit_mean=True, out=None, stream=None, ctx=None, sync=True,
                deterministic=False):
    """Lomb-Scargle power at f0 + k df, k < nf (float64 device tensor);
    deterministic: bitwise-reproducible summation order (slower)."""
    import torch
    t = _dev_f64(t, "t")
    y = _dev_f64(y, "y")
    if dy is not None:
        dy = _dev_f64(dy, "dy")
    if out is None:
        out = torch.empty(int(nf), dtype=torch.float64, device=t.device)
    ctx = ctx or default_context(t.device.index)
    p = make_params(f0, df, nf, eps, precision, normalization, center_data, fit_mean,
                    deterministic)
    fn = load().mils_periodogram if sync else load().mils_periodogram_async
    rc = fn(ctx.handle, ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(y.data_ptr()),
            ctypes.c_void_p(dy.data_ptr()) if dy is not None else None, int(t.numel()),
            ctypes.byref(p), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
    ctx.check(rc)
    return out


def periodogram_noalloc(t, y, dy, f0, df, nf, eps=1e-9, precision="fp64",
                        normalization="standard", center_data=True, fit_mean=True, out=None,
                        stream=None, ctx=None):
    """As periodogram (synchronous), through mils_periodogram_noalloc: the
    library allocates no device memory for the call (its plan tables and
    workspace use a fixed per-GPU scratch).  ``out`` should be given by
    callers that must not allocate either."""
    import torch
    t = _dev_f64(t, "t")
    y = _dev_f64(y, "y")
    if dy is not None:
        dy = _dev_f64(dy, "dy")
    if out is None:
        out = torch.empty(int(nf), dtype=torch.float64, device=t.device)
    ctx = ctx or default_context(t.device.index)
    p = make_params(f0, df, nf, eps, precision, normalization, center_data, fit_mean)
    rc = load().mils_periodogram_noalloc(
        ctx.handle, ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(y.data_ptr()),
        ctypes.c_void_p(dy.data_ptr()) if dy is not None else None, int(t.numel()),
        ctypes.byref(p), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
    ctx.check(rc)
    return out


def context_illposed(ctx=None) -> int:
    """Frequencies whose power was NaN (ill-posed fit) in the context's last
    single-series call whose status has been read."""
    ctx = ctx or default_context()
    return int(load().mils_context_illposed(ctx.handle))


def context_status(ctx=None) -> int:
    ctx = ctx or default_context()
    return load().mils_context_status(ctx.handle)


def autofrequency(t, samples_per_peak=5.0, nyquist_factor=5.0, minimum_frequency=None,
                  maximum_frequency=None):
    """(f0, df, nf) of the automatic frequency grid the paper's benchmarks use
    (Sec. 2: the Astropy default, N_f ~ 12 N_d).  With T the time baseline
    (max t - min t) and N the number of points: the step resolves a peak of
    width 1/T with samples_per_peak frequencies, df = 1 / (samples_per_peak T);
    the grid starts at minimum_frequency (default df / 2) and ends at the
    frequency nearest maximum_frequency on the grid (default nyquist_factor
    times the average Nyquist frequency N / (2 T)).  t: host array or tensor
    (only its extent and length are read)."""
    if hasattr(t, "detach"):
        n = int(t.numel())
        lo, hi = (float(t.min()), float(t.max())) if n else (0.0, 0.0)
    else:
        import numpy as np
        t = np.asarray(t, dtype=np.float64)
        n = int(t.size)
        lo, hi = (float(t.min()), float(t.max())) if n else (0.0, 0.0)
    T = hi - lo
    if n < 2 or not (T > 0.0) or not math.isfinite(T):
        raise ValueError("autofrequency needs at least two distinct finite times")
    if not (samples_per_peak > 0 and nyquist_factor > 0):
        raise ValueError("samples_per_peak and nyquist_factor must be positive")
    df = 1.0 / (samples_per_peak * T)
    f0 = 0.5 * df if minimum_frequency is None else float(minimum_frequency)
    fmax = nyquist_factor * 0.5 * n / T if maximum_frequency is None else float(maximum_frequency)
    if not fmax >= f0:
        raise ValueError("maximum_frequency below minimum_frequency")
    nf = 1 + int(round((fmax - f0) / df))
    return f0, df, nf


def lomb_scargle(t, y, dy=None, samples_per_peak=5.0, nyquist_factor=5.0,
                 minimum_frequency=None, maximum_frequency=None, **kw):
    """The periodogram on the automatic grid of autofrequency: returns
    (f0, df, power), power[k] at f0 + k df (float64 device tensor); kw are
    those of periodogram (eps, precision, normalization, ...)."""
    f0, df, nf = autofrequency(t, samples_per_peak, nyquist_factor, minimum_frequency,
                               maximum_frequency)
    return f0, df, periodogram(t, y, dy, f0, df, nf, **kw)


def trig_sums(t, h, f0, df, nf, eps=1e-9, precision="fp64", stream=None, ctx=None):
    """sum_j h_j exp(+2 pi i (f0 + k df) t_j), k < nf (complex128 device tensor)."""
    import torch
    t = _dev_f64(t, "t")
    h = _dev_f64(h, "h")
    out = torch.empty(2 * int(nf), dtype=torch.float64, device=t.device)
    ctx = ctx or default_context(t.device.index)
    rc = load().mils_trig_sums(ctx.handle, ctypes.c_void_p(t.data_ptr()),
                               ctypes.c_void_p(h.data_ptr()), int(t.numel()), float(f0),
                               float(df), int(nf), float(eps), PRECISIONS[precision],
                               ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
    ctx.check(rc)
    return torch.view_as_complex(out.view(-1, 2))


def periodogram_batch(t, y, dy, nd_off, nf_off, f0, df, eps=1e-9, precision="fp64",
                      normalization="standard", center_data=True, fit_mean=True, out=None,
                      stream=None, ctx=None, return_status=False):
    """Batched periodograms in CSR layout.  t, y, dy: concatenated device
    tensors; nd_off, nf_off: int64 offsets (ncurves + 1, host numpy);
    f0, df: per-curve float64 (host numpy)."""
    import numpy as np
    import torch
    t = _dev_f64(t, "t")
    y = _dev_f64(y, "y")
    if dy is not None:
        dy = _dev_f64(dy, "dy")
    nd_off = np.ascontiguousarray(nd_off, dtype=np.int64)
    nf_off = np.ascontiguousarray(nf_off, dtype=np.int64)
    f0 = np.ascontiguousarray(f0, dtype=np.float64)
    df = np.ascontiguousarray(df, dtype=np.float64)
    nc = nd_off.size - 1
    if out is None:
        out = torch.empty(int(nf_off[-1]), dtype=torch.float64, device=t.device)
    st = np.zeros(nc, dtype=np.int32)
    ctx = ctx or default_context(t.device.index)
    p = make_params(0.0, 1.0, 1, eps, precision, normalization, center_data, fit_mean)
    rc = load().mils_periodogram_batch(
        ctx.handle, nc, nd_off.ctypes.data_as(_I64P), ctypes.c_void_p(t.data_ptr()),
        ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(dy.data_ptr()) if dy is not None else None,
        nf_off.ctypes.data_as(_I64P), f0.ctypes.data_as(_D), df.ctypes.data_as(_D),
        ctypes.byref(p), ctypes.c_void_p(out.data_ptr()),
        st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _stream_ptr(stream))
    if rc not in (MILS_OK, MILS_ERR_INVALID_ARG, MILS_ERR_DEGENERATE) or not return_status:
        ctx.check(rc)
    return (out, st) if return_status else out


def direct_periodogram(t, y, dy, f0, df, nf, normalization="standard", center_data=True,
                       fit_mean=True, out=None, stream=None, ctx=None):
    """The periodogram by direct FP64 summation over the points at every
    frequency (float64 device tensor of nf values)."""
    import torch
    t = _dev_f64(t, "t")
    y = _dev_f64(y, "y")
    if dy is not None:
        dy = _dev_f64(dy, "dy")
    if out is None:
        out = torch.empty(int(nf), dtype=torch.float64, device=t.device)
    ctx = ctx or default_context(t.device.index)
    p = make_params(f0, df, nf, 1e-9, "fp64", normalization, center_data, fit_mean)
    rc = load().mils_direct_periodogram(
        ctx.handle, ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(y.data_ptr()),
        ctypes.c_void_p(dy.data_ptr()) if dy is not None else None, int(t.numel()),
        ctypes.byref(p), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
    ctx.check(rc)
    return out


def direct_trig_sums(t, h, f0, df, nf, stream=None, ctx=None):
    """sum_j h_j exp(+2 pi i (f0 + k df) t_j), k < nf, by direct FP64 summation
    (complex128 device tensor)."""
    import torch
    t = _dev_f64(t, "t")
    h = _dev_f64(h, "h")
    out = torch.empty(2 * int(nf), dtype=torch.float64, device=t.device)
    ctx = ctx or default_context(t.device.index)
    rc = load().mils_direct_trig_sums(ctx.handle, ctypes.c_void_p(t.data_ptr()),
                                      ctypes.c_void_p(h.data_ptr()), int(t.numel()), float(f0),
                                      float(df), int(nf), ctypes.c_void_p(out.data_ptr()),
                                      _stream_ptr(stream))
    ctx.check(rc)
    return torch.view_as_complex(out.view(-1, 2))


def periodogram_shared_t(t, y, dy, f0, df, nf, eps=1e-9, precision="fp64",
                         normalization="standard", center_data=True, fit_mean=True, out=None,
                         stream=None, ctx=None, return_status=False):
    """Periodograms of the rows of y (nseries x nd device tensor), all observed
    at times t (nd).  dy: None, one row of nd shared by every series, or
    nseries x nd.  Returns an nseries x nf float64 device tensor."""
    import numpy as np
    import torch
    t = _dev_f64(t, "t")
    y = _dev_f64(y, "y")
    nd = int(t.numel())
    if y.dim() != 2 or y.shape[1] != nd:
        raise ValueError("y must be nseries x nd")
    ns = int(y.shape[0])
    stride = 0
    if dy is not None:
        dy = _dev_f64(dy, "dy")
        if dy.dim() == 2 and dy.shape[0] == ns and ns > 1:
            stride = nd
        if dy.shape[-1] != nd or (dy.dim() == 2 and dy.shape[0] not in (1, ns)):
            raise ValueError("dy must be nd, 1 x nd or nseries x nd")
    if out is None:
        out = torch.empty((ns, int(nf)), dtype=torch.float64, device=t.device)
    st = np.zeros(ns, dtype=np.int32)
    ctx = ctx or default_context(t.device.index)
    p = make_params(f0, df, nf, eps, precision, normalization, center_data, fit_mean)
    rc = load().mils_periodogram_shared_t(
        ctx.handle, ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(y.data_ptr()),
        ctypes.c_void_p(dy.data_ptr()) if dy is not None else None, stride, nd, ns,
        ctypes.byref(p), ctypes.c_void_p(out.data_ptr()),
        st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _stream_ptr(stream))
    if rc not in (MILS_OK, MILS_ERR_INVALID_ARG, MILS_ERR_DEGENERATE) or not return_status:
        ctx.check(rc)
    return (out, st) if return_status else out


def pack_curves(curves, device=None, with_dy=True):
    """CSR packing of a list of workloads.Curve for periodogram_batch:
    returns (t, y, dy, nd_off, nf_off, f0, df) with device tensors for the data."""
    import numpy as np
    import torch
    nd = np.array([c.t.size for c in curves], dtype=np.int64)
    nf = np.array([c.nf for c in curves], dtype=np.int64)
    nd_off = np.concatenate([[0], np.cumsum(nd)]).astype(np.int64)
    nf_off = np.concatenate([[0], np.cumsum(nf)]).astype(np.int64)
    dev = device or torch.device("cuda", torch.cuda.current_device())
    cat = lambda xs: torch.from_numpy(np.ascontiguousarray(np.concatenate(xs), dtype=np.float64)).to(dev)  # noqa: E731
    t = cat([c.t for c in curves])
    y = cat([c.y for c in curves])
    dy = cat([c.dy for c in curves]) if with_dy else None
    f0 = np.array([c.f0 for c in curves], dtype=np.float64)
    df = np.array([c.df for c in curves], dtype=np.float64)
    return t, y, dy, nd_off, nf_off, f0, df


def split_power(power, nf_off):
    """Per-series numpy views of a batched power tensor."""
    p = power.cpu().numpy()
    return [p[nf_off[i]:nf_off[i + 1]] for i in range(len(nf_off) - 1)]


class Server:
    """Serving loop on one device (mils_server_*): submit host arrays, get
    tickets, wait and take host results."""

    def __init__(self, device=0, hbm_budget_bytes=0, lanes=0, max_batch=0, queue_capacity=0,
                 tick_us=0):
        lib = load()
        cfg = mils_server_config(int(hbm_budget_bytes), int(lanes), int(max_batch),
                                 int(queue_capacity), int(tick_us))
        h = _P()
        rc = lib.mils_server_create(int(device), ctypes.byref(cfg), ctypes.byref(h))
        if rc != MILS_OK:
            raise MilsError(rc, "mils_server_create failed")
        self.handle = h

    def submit(self, t, y, dy, f0, df, nf, eps=1e-9, precision="fp64",
               normalization="standard", center_data=True, fit_mean=True):
        """Returns (status, ticket); status is MILS_OK, MILS_ERR_BUSY, ..."""
        import numpy as np
        t = np.ascontiguousarray(t, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        dyp = None
        if dy is not None:
            dy = np.ascontiguousarray(dy, dtype=np.float64)
            dyp = dy.ctypes.data
        req = mils_request(t.ctypes.data, y.ctypes.data, dyp, t.size,
                           make_params(f0, df, nf, eps, precision, normalization, center_data,
                                       fit_mean))
        tk = ctypes.c_uint64()
        rc = load().mils_server_submit(self.handle, ctypes.byref(req), ctypes.byref(tk))
        return rc, tk.value

    def warm(self, nf_max, eps=1e-9, precision="fp64", normalization="standard",
             center_data=True, fit_mean=True):
        """Build every lane's plans of the classes up to nf_max (blocking)."""
        p = make_params(0.01, 0.01, int(nf_max), eps, precision, normalization, center_data,
                        fit_mean)
        return load().mils_server_warm(self.handle, ctypes.byref(p), int(nf_max))

    def poll(self, ticket):
        st = ctypes.c_int32()
        rc = load().mils_server_poll(self.handle, ticket, ctypes.byref(st))
        return rc, st.value

    def wait(self, ticket, timeout_us=-1):
        return load().mils_server_wait(self.handle, ticket, int(timeout_us))

    def take(self, ticket, nf):
        """(status, power numpy array or None, stats dict)."""
        import numpy as np
        out = np.empty(int(nf))
        st = mils_request_stats()
        rc = load().mils_server_take(self.handle, ticket, out.ctypes.data, ctypes.byref(st))
        stats = {"submit_s": st.submit_s, "start_s": st.start_s, "done_s": st.done_s,
                 "status": st.status, "batch_size": st.batch_size}
        return rc, (out if rc == MILS_OK else None), stats

    def stats(self) -> dict:
        c = mils_server_counters()
        rc = load().mils_server_stats(self.handle, ctypes.byref(c))
        if rc != MILS_OK:
            raise MilsError(rc, "mils_server_stats failed")
        return {f: getattr(c, f) for f, _ in mils_server_counters._fields_}

    def last_error(self) -> str:
        """Message of the first device error that stopped a lane ("" if none)."""
        return load().mils_server_last_error(self.handle).decode()

    def close(self):
        if self.handle:
            load().mils_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
