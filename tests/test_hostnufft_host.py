"""The plain host FP64 NUFFT baseline (hostnufft/) against the oracle (CPU).

The host NUFFT is the CPU baseline the benchmark times beside the GPU path
(the paper's CPU backend, Sec. 2 and Sec. 2.1); these tests hold it to the
same parity bar as the GPU path: max|P - P_ref| / max|P_ref| <= 1e-8 at
eps = 1e-9 (FP64).  Its FFT is checked against numpy's (a library special
case of the transform it computes).
"""
import numpy as np
import pytest

import hostnufft
import oracle
from paper_2409_08090_amd import workloads


def _err(p, ref):
    return float(np.max(np.abs(p - ref)) / np.max(np.abs(ref)))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 16, 60, 96, 1000, 4096, 15000, 46875, 131072])
def test_host_fft_matches_numpy(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = np.fft.ifft(x) * n  # sum_l x_l exp(+2 pi i l m / n)
    got = hostnufft.fft(x, threads=4)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_small_curve_full_grid():
    c = workloads.single_small(seed=0)
    p = hostnufft.periodogram(c.t, c.y, c.dy, c.f0, c.df, c.nf, eps=1e-9, threads=4)
    ref = oracle.periodogram(c.t, c.y, c.dy, c.f0, c.df, nf=c.nf)
    assert _err(p, ref) <= 1e-8


def test_noiseless_sinusoid_power_one():
    c = workloads.single_small(seed=0, noiseless=True)
    p = hostnufft.periodogram(c.t, c.y, c.dy, c.f0, c.df, c.nf, eps=1e-9, threads=4)
    assert abs(p[184] - 1.0) <= 1e-8


def test_shrunk_large_curve_sampled():
    # the large-curve recipe (gapped seasons, three sinusoids, dy ~ U(0.1, 0.3))
    # at N_d = 2e4, N_f = 2.4e5, on sampled frequencies incl. both band edges
    c = workloads.single_large(seed=1, nd=20000, span_years=2)
    p = hostnufft.periodogram(c.t, c.y, c.dy, c.f0, c.df, c.nf, eps=1e-9, threads=4)
    rng = np.random.default_rng(2)
    k = np.unique(np.concatenate([rng.integers(0, c.nf, 2000), np.arange(0, 200),
                                  np.arange(c.nf - 200, c.nf), [int(np.argmax(p))]]))
    ref = oracle.periodogram(c.t, c.y, c.dy, c.f0, c.df, k=k)
    assert _err(p[k], ref) <= 1e-8


def test_unsorted_times_and_unit_weights():
    c = workloads.single_small(seed=7, nd=700, nf=5000)
    perm = np.random.default_rng(1).permutation(c.nd)
    p = hostnufft.periodogram(c.t[perm], c.y[perm], None, c.f0, c.df, c.nf, eps=1e-9, threads=4)
    ref = oracle.periodogram(c.t, c.y, None, c.f0, c.df, nf=c.nf)
    assert _err(p, ref) <= 1e-8


def test_batch_matches_oracle_per_series():
    curves = workloads.batch(seed=3, ncurves=12, nd_min=100, nd_max=2000)
    out, st = hostnufft.batch(curves, eps=1e-9, threads=4)
    assert np.all(st == 0)
    off = 0
    for c in curves:
        ref = oracle.periodogram(c.t, c.y, c.dy, c.f0, c.df, nf=c.nf)
        assert _err(out[off:off + c.nf], ref) <= 1e-8
        off += c.nf
