"""GPU direct evaluation (every sum term by term in FP64, the paper's
brute-force method) pinned against the CPU oracle, then used to check the
transform path at every frequency of the full-size curve.

The direct kernel and the oracle compute the same exact function up to FP64
rounding (both reduce the phases in double-double), so they must agree far
below the transform's tolerance:
  periodogram: max|P - P_ref| / max|P_ref| <= 1e-10
  raw sums:    max|g - g_ref| <= 1e-12 sum_j |h_j|
The transform path is then held to its own tolerances against the direct
result at all N_f = 1.2e7 frequencies (1e-8 in FP64 at eps = 1e-9, 1e-4 in
FP32 at eps = 1e-5), where the oracle can only sample.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import oracle  # noqa: E402
from paper_2409_08090_amd import mils, workloads  # noqa: E402


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def rel_err(p, ref):
    return np.max(np.abs(p - ref)) / np.max(np.abs(ref))


def direct(c, dy=True, **kw):
    p = mils.direct_periodogram(dev(c.t), dev(c.y), dev(c.dy) if dy else None, c.f0, c.df, c.nf,
                                **kw)
    torch.cuda.synchronize()
    return p.cpu().numpy()


def test_direct_matches_oracle_small():
    c = workloads.single_small(seed=0)
    p = direct(c)
    ref = oracle.periodogram(c.t, c.y, c.dy, c.f0, c.df, nf=c.nf)
    err = rel_err(p, ref)
    print(f"[direct single_small] max-normalised {err:.3e}", flush=True)
    assert err <= 1e-10


def test_direct_noiseless_sinusoid_power_is_one():
    c = workloads.single_small(seed=0, noiseless=True)
    assert abs(direct(c)[184] - 1.0) < 1e-10


@pytest.mark.parametrize("normalization", ["standard", "model", "log", "psd"])
@pytest.mark.parametrize("center_data,fit_mean", [(True, True), (False, False)])
def test_direct_normalizations(normalization, center_data, fit_mean):
    c = workloads.uniform_series(seed=31, nd=600, nf=3000, span=40.0)
    c.y = c.y + 1.7
    p = direct(c, normalization=normalization, center_data=center_data, fit_mean=fit_mean)
    ref = oracle.periodogram(c.t, c.y, c.dy, c.f0, c.df, nf=c.nf, normalization=normalization,
                             center_data=center_data, fit_mean=fit_mean)
    assert rel_err(p, ref) <= 1e-10


@pytest.mark.parametrize("nd,nf", [(3, 1), (255, 4095), (257, 4097), (1000, 9000)])
def test_direct_ragged_sizes_unit_weights(nd, nf):
    c = workloads.uniform_series(seed=32 + nd, nd=nd, nf=nf, span=10.0, sorted_t=False)
    p = direct(c, dy=False)
    ref = oracle.periodogram(c.t, c.y, None, c.f0, c.df, nf=c.nf)
    assert rel_err(p, ref) <= (1e-8 if nd < 10 else 1e-10)


def test_direct_single_point_is_degenerate():
    c = workloads.uniform_series(seed=35, nd=1, nf=5)
    with pytest.raises(mils.MilsError) as e:
        direct(c)
    assert e.value.status == mils.MILS_ERR_DEGENERATE


def test_direct_raw_sums_match_oracle():
    rng = np.random.default_rng(33)
    t = np.sort(rng.uniform(0.0, 2000.0, 700))
    h = rng.normal(0.0, 1.0, 700)
    f0, df, nf = -3.1, 0.0137, 5000
    g = mils.direct_trig_sums(dev(t), dev(h), f0, df, nf).cpu().numpy()
    ref = oracle.trig_sums(t, h, f0, df, nf=nf)
    assert np.max(np.abs(g - ref)) <= 1e-12 * np.sum(np.abs(h))


def test_direct_constant_data_is_degenerate():
    c = workloads.uniform_series(seed=34, nd=100, nf=50)
    c.y[:] = 2.0
    with pytest.raises(mils.MilsError) as e:
        direct(c)
    assert e.value.status == mils.MILS_ERR_DEGENERATE


@pytest.fixture(scope="module")
def large_direct():
    """The full-size curve and its direct periodogram (computed once)."""
    import time
    c = workloads.single_large(seed=1)
    t, y, dy = dev(c.t), dev(c.y), dev(c.dy)
    mils.direct_periodogram(t, y, dy, c.f0, c.df, 4096)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref = mils.direct_periodogram(t, y, dy, c.f0, c.df, c.nf)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    print(f"[direct full size] {sec:.2f} s, {c.nd * c.nf / sec:.3e} sums/s", flush=True)
    return c, (t, y, dy), ref.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_transform_matches_direct_at_every_frequency_full_size(precision, large_direct):
    c, (t, y, dy), ref = large_direct
    eps = {"fp64": 1e-9, "fp32": 1e-5}[precision]
    p = mils.periodogram(t, y, dy, c.f0, c.df, c.nf, eps=eps, precision=precision)
    torch.cuda.synchronize()
    p = p.cpu().numpy()
    err = rel_err(p, ref)
    r = np.abs(p - ref) / np.maximum(np.abs(ref), 1e-300)
    print(f"[transform vs direct, all {c.nf} frequencies, {precision}] max-normalised "
          f"{err:.3e}  median {np.median(r):.3e}  p99 {np.percentile(r, 99):.3e}", flush=True)
    assert err <= {"fp64": 1e-8, "fp32": 1e-4}[precision]


def test_direct_full_size_matches_oracle_sampled(large_direct):
    c, _, ref = large_direct
    rng = np.random.default_rng(9)
    k = np.unique(np.concatenate([rng.integers(0, c.nf, 100), np.arange(30),
                                  np.arange(c.nf - 30, c.nf), np.argsort(ref)[-20:]]))
    o = oracle.periodogram(c.t, c.y, c.dy, c.f0, c.df, k=k)
    err = rel_err(ref[k], o)
    print(f"[direct full size vs oracle] {k.size} frequencies, max-normalised {err:.3e}",
          flush=True)
    assert err <= 1e-10
