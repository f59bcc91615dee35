"""Host-side tests of the C ABI (no GPU): the library loads and exports every
symbol of include/mils.h, argument validation returns the documented codes,
and the planner's choices satisfy their invariants."""
import ctypes
import math

import numpy as np
import os
import re

import pytest

from paper_2409_08090_amd import mils

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"^[A-Za-z_][\w \*]*?\b(mils_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = mils.load()
    names = header_functions()
    assert "mils_periodogram" in names and "mils_trig_sums" in names
    for n in names:
        assert hasattr(lib, n), f"{n} declared in include/ but not exported"
    # and the binding knows each of them
    assert set(names) <= set(mils.SIGNATURES), set(names) - set(mils.SIGNATURES)


def test_version_and_status_strings():
    assert mils.version() == 10000
    assert mils.status_str(0) == "ok"
    assert "invalid" in mils.status_str(-1)


@pytest.fixture
def host_ctx():
    c = mils.Context(-1)
    yield c
    c.close()


def _check(t, y, nd, p, power):
    return mils.load().mils_check_periodogram_args(t, y, nd, ctypes.byref(p) if p else None, power)


def test_argument_validation_codes():
    ok = mils.make_params(0.01, 0.01, 100)
    P = ctypes.c_void_p(16)  # any non-null pointer: nothing is dereferenced
    assert _check(P, P, 10, ok, P) == mils.MILS_OK
    assert _check(None, P, 10, ok, P) == mils.MILS_ERR_INVALID_ARG
    assert _check(P, None, 10, ok, P) == mils.MILS_ERR_INVALID_ARG
    assert _check(P, P, 10, ok, None) == mils.MILS_ERR_INVALID_ARG
    assert _check(P, P, 0, ok, P) == mils.MILS_ERR_INVALID_ARG
    assert _check(P, P, 2 ** 31, ok, P) == mils.MILS_ERR_INVALID_ARG
    assert _check(P, P, 10, None, P) == mils.MILS_ERR_INVALID_ARG
    bad = [
        mils.make_params(0.01, 0.0, 100),
        mils.make_params(0.01, -1.0, 100),
        mils.make_params(float("nan"), 0.01, 100),
        mils.make_params(0.01, float("inf"), 100),
        mils.make_params(0.01, 0.01, 0),
    ]
    for p in bad:
        assert _check(P, P, 10, p, P) == mils.MILS_ERR_INVALID_ARG
    p = mils.make_params(0.01, 0.01, 100)
    p.precision = 7
    assert _check(P, P, 10, p, P) == mils.MILS_ERR_INVALID_ARG
    p = mils.make_params(0.01, 0.01, 100)
    p.normalization = 9
    assert _check(P, P, 10, p, P) == mils.MILS_ERR_INVALID_ARG
    p = mils.make_params(0.01, 0.01, 100)
    p.flags = 8
    assert _check(P, P, 10, p, P) == mils.MILS_ERR_INVALID_ARG
    # the reproducible mode is a valid flag
    assert _check(P, P, 10, mils.make_params(0.01, 0.01, 100, deterministic=True), P) == mils.MILS_OK
    # tolerance outside the precision's range, or too many frequencies
    assert _check(P, P, 10, mils.make_params(0.01, 0.01, 100, eps=1e-15), P) == mils.MILS_ERR_UNSUPPORTED
    assert _check(P, P, 10, mils.make_params(0.01, 0.01, 100, eps=1e-7, precision="fp32"),
                  P) == mils.MILS_ERR_UNSUPPORTED
    assert _check(P, P, 10, mils.make_params(0.01, 0.01, 100, eps=0.5), P) == mils.MILS_ERR_UNSUPPORTED
    assert _check(P, P, 10, mils.make_params(0.01, 0.01, 2 ** 28 + 1), P) == mils.MILS_ERR_UNSUPPORTED


def test_host_only_context_refuses_compute(host_ctx):
    lib = mils.load()
    p = mils.make_params(0.01, 0.01, 100)
    P = ctypes.c_void_p(16)
    rc = lib.mils_periodogram(host_ctx.handle, P, P, None, 10, ctypes.byref(p), P, None)
    assert rc == mils.MILS_ERR_DEVICE
    rc = lib.mils_trig_sums(host_ctx.handle, P, P, 10, 0.0, 0.1, 10, 1e-9, 0, P, None)
    assert rc == mils.MILS_ERR_DEVICE
    # invalid arguments are rejected before the device is considered
    rc = lib.mils_periodogram(host_ctx.handle, None, P, None, 10, ctypes.byref(p), P, None)
    assert rc == mils.MILS_ERR_INVALID_ARG
    assert lib.mils_periodogram(None, P, P, None, 10, ctypes.byref(p), P, None) == \
        mils.MILS_ERR_INVALID_ARG


def _smooth(n):
    for f in (2, 3, 5):
        while n % f == 0:
            n //= f
    return n == 1


@pytest.mark.parametrize("nf,eps,prec", [
    (12_000, 1e-9, "fp64"), (12_000_000, 1e-9, "fp64"), (12_000_000, 1e-5, "fp32"),
    (1, 1e-9, "fp64"), (7, 1e-9, "fp64"), (1200, 1e-5, "fp32"), (120_000, 1e-9, "fp64"),
    (2 ** 28, 1e-9, "fp64"), (999_983, 1e-6, "fp32"), (240_000, 1e-12, "fp64"),
])
def test_planner_invariants(nf, eps, prec):
    d = mils.plan_info(nd=1000, nf=nf, eps=eps, precision=prec)
    n = d["n"]
    assert n >= math.ceil(1.25 * nf) - 1  # sigma 1.25 in both precisions
    assert _smooth(n)
    assert math.prod(d["len"]) == n
    assert 1 <= d["npass"] <= 4
    assert 2 <= d["width"] <= 20
    # the ES aliasing estimate exp(-pi w sqrt(1 - 1/sigma)) meets the tolerance
    margin = 8 if prec == "fp64" else 2
    assert math.exp(-math.pi * d["width"] * math.sqrt(1 - 1 / d["sigma"])) <= eps / margin * 1.0001
    assert n % d["tile"] == 0 and d["tile"] <= 1024
    assert 1 <= d["last_rows"] <= 8 and 0 < d["last_lds_bytes"] <= 163840


def _tw2(L):
    return 64 + (L + 63) // 64


def _check_fft2_plan(d, prec):
    # two-pass register-tile plans: lines of 2048..8192 (three grids: last
    # line at most 4096), workgroups of at most 1024 threads (16 elements
    # each), LDS of the exchange lines (one half at a time in FP64: 8 bytes
    # per element), the two-level twiddle table and (last pass) the other
    # grids' results, within 160 KB
    elem = 16 if prec == "fp64" else 8
    L0, L1 = d["len"]
    assert d["npass"] == 2 and d["n"] == L0 * L1, d
    assert L0 in (2048, 4096, 8192) and L1 in (2048, 4096), d
    C = d["first_cols"]
    assert C == min(8, 16384 // L0) and C * L0 // 16 <= 1024 and 3 * L1 // 16 <= 1024, d
    # first-pass lines are 16/C elements apart modulo 16 (distinct LDS bank
    # pairs for the lanes of one access cycle); last-pass lines pad by 8
    lp_first = lambda L: L + L // 16 + (16 // C if C >= 2 else 8)  # noqa: E731
    lp = lambda L: L + L // 16 + 8  # noqa: E731
    assert d["first_lds_bytes"] == C * lp_first(L0) * 8 + _tw2(L0) * elem <= 163840, d
    if prec == "fp64":  # three grids side by side, exchanged and gathered in halves
        last = max(3 * lp(L1) * 8, 3 * (L1 // 2) * elem) + _tw2(L1) * elem
    else:  # the three grids one after another through one exchange line
        last = lp(L1) * 8 + _tw2(L1) * elem
    assert d["last_lds_bytes"] == last <= 163840, d


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fft_passes_fit_one_workgroup_over_a_size_sweep(prec):
    # LDS of a workgroup: last pass L * 3D elements + twiddles, first pass
    # L * C elements + twiddles + L row flags; twiddles are L entries, or the
    # two-level table of big passes (1024 threads, up to 160 KB of LDS)
    elem = 16 if prec == "fp64" else 8
    for nf in sorted({int(x) for x in np.geomspace(1, 3e7, 300)}):
        d = mils.plan_info(nd=1000, nf=nf, eps=1e-9 if prec == "fp64" else 1e-5, precision=prec)
        if d["fft2"]:
            _check_fft2_plan(d, prec)
            continue
        L, D, big = d["len"][-1], d["last_rows"], d["big"]
        cap, emax = (163840, 9600 if prec == "fp64" else 19200) if big else \
            (65536, 3072 if prec == "fp64" else 6144)
        ntw = _tw2(L) if big else L
        assert d["last_lds_bytes"] == elem * (L * 3 * D + ntw) <= cap, (nf, d)
        assert 3 * D * L <= emax, (nf, d)
        if d["npass"] > 1:
            L0, C = d["len"][0], d["first_cols"]
            assert C & (C - 1) == 0 and (not big or C >= (2 if prec == "fp64" else 4)), (nf, d)
            assert d["first_lds_bytes"] == elem * (L0 * C + (_tw2(L0) if big else L0)) + L0 + 16
            assert d["first_lds_bytes"] <= cap and L0 * C <= (emax if big else emax * 2 // 3), (nf, d)
        if big:
            assert d["npass"] == 2


def test_large_curve_plans():
    # the N_f = 1.2e7 curve: the two-pass register-tile FFT on a 4096 x 4096
    # grid by default; without it three small LDS passes, or (on request)
    # two big ones
    import subprocess, sys
    for prec, eps in (("fp64", 1e-9), ("fp32", 1e-5)):
        d = mils.plan_info(nd=1_000_000, nf=12_000_000, eps=eps, precision=prec)
        assert d["npass"] == 2 and d["fft2"] == 1 and d["len"] == [4096, 4096], d
        _check_fft2_plan(d, prec)
    code = ("from paper_2409_08090_amd import mils; "
            "d = mils.plan_info(1_000_000, 12_000_000, 1e-9); print(d['npass'], d['big'], d['fft2'])")
    for env, want in (({"MILS_FFT2": "0"}, ["3", "0", "0"]),
                      ({"MILS_FFT2": "0", "MILS_FFT_BIG": "1"}, ["2", "1", "0"])):
        out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                             env={**os.environ, **env}, check=True).stdout.split()
        assert out == want, (env, out)


def test_kernel_error_estimate_falls_with_tolerance():
    est = []
    for eps in (1e-3, 1e-6, 1e-9, 1e-12, 1e-14):
        d = mils.plan_info(1000, 100_000, eps)
        est.append(math.exp(-math.pi * d["width"] * math.sqrt(1 - 1 / d["sigma"])))
    assert est == sorted(est, reverse=True) and est[0] > 100 * est[-1]
    # at fixed sigma the width grows as the tolerance shrinks
    ws = [mils.plan_info(1000, 100_000, eps)["width"] for eps in (1e-3, 1e-6, 1e-9)]
    assert ws == sorted(ws) and ws[0] < ws[-1]


def test_large_curve_grid_and_width():
    # the planner may trade a slightly larger grid (sigma up to ~1.3 x 1.25)
    # for fewer radix stages and a narrower kernel; the width still meets eps
    d = mils.plan_info(nd=1_000_000, nf=12_000_000, eps=1e-9)
    assert 15_000_000 <= d["n"] <= 1.3 * 15_000_000
    w, sigma = d["width"], d["sigma"]
    assert math.exp(-math.pi * w * math.sqrt(1 - 1 / sigma)) <= 1e-9 / 8 * 1.0001
    assert math.exp(-math.pi * (w - 1) * math.sqrt(1 - 1 / sigma)) > 1e-9 / 8  # no wider than needed
    assert math.prod(d["len"]) == d["n"]


def test_server_config_and_device_checks():
    lib = mils.load()
    h = ctypes.c_void_p()
    bad = mils.mils_server_config(0, 99, 0, 0, 0)
    assert lib.mils_server_create(0, ctypes.byref(bad), ctypes.byref(h)) == mils.MILS_ERR_INVALID_ARG
    assert lib.mils_server_create(-1, None, ctypes.byref(h)) == mils.MILS_ERR_DEVICE
    assert lib.mils_server_create(0, None, None) == mils.MILS_ERR_INVALID_ARG
    assert lib.mils_server_submit(None, None, None) == mils.MILS_ERR_INVALID_ARG
    assert lib.mils_server_destroy(None) == mils.MILS_ERR_INVALID_ARG
    assert lib.mils_server_last_error(None) == b""


def test_graph_switch_on_host_context():
    lib = mils.load()
    assert lib.mils_context_set_graphs(None, 0) == mils.MILS_ERR_INVALID_ARG
    ctx = mils.Context(-1)  # host-only: nothing to release
    ctx.set_graphs(False)
    ctx.set_graphs(True)
    ctx.close()


@pytest.mark.parametrize("nf,eps,prec", [(12_000_000, 1e-9, "fp64"), (100_000, 1e-12, "fp64"),
                                         (100_000, 1e-6, "fp64"), (1000, 1e-9, "fp64"),
                                         (12_000_000, 1e-5, "fp32"), (5000, 1e-3, "fp32")])
def test_kernel_polynomials_reproduce_the_es_kernel(nf, eps, prec):
    # The spread evaluates phi(z) = exp(beta (sqrt(1 - z^2) - 1)) at the w cells of
    # a point from per-cell polynomials; here they are checked against phi itself.
    coef, w, beta = mils.kernel_table(nf, eps, prec)
    nc, kmax = coef.shape
    assert kmax >= w and not np.any(coef[:, w:])
    t = np.linspace(0.0, 1.0, 1001, endpoint=False)
    u = 2 * t - 1
    worst = 0.0
    for k in range(w):
        acc = np.zeros_like(u)
        for j in range(nc):
            acc = acc * u + coef[j, k]
        z = (k + t) / (w / 2) - 1
        ref = np.exp(beta * (np.sqrt(np.maximum(1 - z * z, 0.0)) - 1))
        worst = max(worst, np.max(np.abs(acc - ref)))
    # limited by the kink of phi at |z| = 1, of size exp(-beta), and by rounding
    bound = 4 * math.exp(-beta) + (1e-13 if prec == "fp64" else 1e-7)
    assert worst <= bound, (w, beta, worst, bound)
    # and well below the tolerance the plan was made for
    assert worst <= eps / 10


def test_batch_tuning_query_without_a_decision():
    ctx = mils.Context(-1)
    assert ctx.batch_tuning(12_000, 1e-9, "fp64") is None
    lib = mils.load()
    import ctypes as C
    sg, tm = C.c_double(), C.c_int32()
    assert lib.mils_batch_tuning(ctx.handle, 0, 1e-9, 0, C.byref(sg), C.byref(tm)) == mils.MILS_ERR_INVALID_ARG
    ctx.close()


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
@pytest.mark.parametrize("nf,eps,prec", [(12_000, 1e-9, "fp64"), (12_000_000, 1e-9, "fp64"),
                                         (100_000, 1e-12, "fp64"), (12_000_000, 1e-5, "fp32"),
                                         (7, 1e-9, "fp64")])
def test_kernel_transform_matches_adaptive_quadrature(nf, eps, prec):
    # 1/phihat(m) = 1 / (w int_0^1 phi(z) cos(pi w m z / n) dz) by the plan's
    # Gauss-Legendre rule, against scipy's adaptive quadrature of the same
    # integral (an independent rule): the deconvolution of Sec. 1, Eq. 2.
    from scipy import integrate
    K = nf // 2
    modes = np.unique(np.array([0, 1, 2, K // 3, K // 2, max(K - 1, 0), K], dtype=np.int64))
    inv, n = mils.kernel_transform(nf, modes, eps, prec)
    _, w, beta = mils.kernel_table(nf, eps, prec)
    phat0 = None
    for m, v in zip(modes, inv):
        a = math.pi * w * m / n
        f = lambda z: math.exp(beta * (math.sqrt(max(1.0 - z * z, 0.0)) - 1.0)) * math.cos(a * z)  # noqa: E731
        val, _ = integrate.quad(f, 0.0, 1.0, limit=400, epsabs=1e-300, epsrel=1e-12)
        ref = w * val  # phihat(m)
        phat0 = ref if m == 0 else phat0
        # the rule's error comes from the kink of phi at z = 1 (size exp(-beta)),
        # relative to phihat(0): 1e-12 for the FP64 plans, ~1e-10 for the FP32
        # plan's narrow kernel
        bound = (1e-12 + 1e-3 * math.exp(-beta)) * phat0
        assert abs(1.0 / v - ref) <= bound, (m, 1.0 / v, ref, bound)
    # the deconvolution grows towards the band edge (the kernel's transform decays)
    assert np.all(np.diff(inv) > 0)
