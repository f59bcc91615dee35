"""The allocation-free periodogram (mils_periodogram_noalloc) against
mils_periodogram through the C ABI (GPU): two calls in a row, the second
with a smaller input, in FP64 and FP32; both paths agree to rounding and
match the oracle within the path's tolerance.  A call too large for the
scratch is refused without touching the device and leaves the context
usable."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import oracle  # noqa: E402
from paper_2409_08090_amd import mils, workloads  # noqa: E402

EPS = {"fp64": 1e-9, "fp32": 1e-5}
TOL = {"fp64": 1e-8, "fp32": 1e-4}


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def rel(p, ref):
    return float(np.max(np.abs(p - ref)) / np.max(np.abs(ref)))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_matches_periodogram_on_two_calls(precision):
    ctx = mils.Context(0)
    cases = [workloads.single_large(seed=21, nd=40_000, span_years=3),   # three-pass plan
             workloads.single_small(seed=22, nd=700, nf=8000)]            # smaller input
    for c in cases:
        t, y, dy = dev(c.t), dev(c.y), dev(c.dy)
        out = torch.full((c.nf,), -1.0, dtype=torch.float64, device="cuda")
        mils.periodogram_noalloc(t, y, dy, c.f0, c.df, c.nf, eps=EPS[precision],
                                 precision=precision, out=out, ctx=ctx)
        got = out.cpu().numpy()
        ref_path = mils.periodogram(t, y, dy, c.f0, c.df, c.nf, eps=EPS[precision],
                                    precision=precision, ctx=ctx).cpu().numpy()
        assert rel(got, ref_path) <= (1e-12 if precision == "fp64" else 1e-6), (c.nd, c.nf)
        k = np.unique(np.concatenate([np.arange(min(c.nf, 400)),
                                      np.random.default_rng(c.nd).integers(0, c.nf, 400)]))
        ref = oracle.periodogram(c.t, c.y, c.dy, c.f0, c.df, k=k)
        assert rel(got[k], ref) <= TOL[precision], (c.nd, c.nf)
    ctx.close()


def test_noalloc_refuses_a_call_larger_than_its_scratch():
    ctx = mils.Context(0)
    c = workloads.single_small(seed=23)
    t, y, dy = dev(c.t), dev(c.y), dev(c.dy)
    big_nf = 4_000_000
    out = torch.empty(big_nf, dtype=torch.float64, device="cuda")
    with pytest.raises(mils.MilsError) as e:
        mils.periodogram_noalloc(t, y, dy, c.f0, c.df, big_nf, out=out, ctx=ctx)
    assert e.value.status == mils.MILS_ERR_UNSUPPORTED
    # the context still computes, through both entry points
    p1 = mils.periodogram_noalloc(t, y, dy, c.f0, c.df, c.nf, ctx=ctx).cpu().numpy()
    p2 = mils.periodogram(t, y, dy, c.f0, c.df, c.nf, ctx=ctx).cpu().numpy()
    assert rel(p1, p2) <= 1e-12
    ctx.close()
