"""Calls captured into a caller's HIP graph (GPU).

A captured call may only use the plan tables and workspace that an earlier
uncaptured call of the same sizes left on the context: otherwise it is
refused with MILS_ERR_BUSY and the context stays usable.  Once a call has
been captured, a later workspace growth keeps the captured buffer, so the
caller's graph still replays to the eager result.
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


def _capture(ctx, c, t, y, dy, out, sync=False):
    """Capture one periodogram call; returns (graph, status of the call)."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    status = mils.MILS_OK
    with torch.cuda.graph(g, stream=s):
        try:
            mils.periodogram(t, y, dy, c.f0, c.df, c.nf, out=out, ctx=ctx, sync=sync,
                             stream=torch.cuda.current_stream())
        except mils.MilsError as e:
            status = e.status
    return g, status


def test_captured_call_without_plan_or_workspace_is_refused():
    c = workloads.single_small(seed=0)
    t, y, dy = dev(c.t), dev(c.y), dev(c.dy)
    out = torch.empty(c.nf, dtype=torch.float64, device="cuda")
    ctx = mils.Context(0)
    # no plan yet
    g, st = _capture(ctx, c, t, y, dy, out)
    assert st == mils.MILS_ERR_BUSY
    del g
    # a synchronous call cannot be captured
    g, st = _capture(ctx, c, t, y, dy, out, sync=True)
    assert st == mils.MILS_ERR_INVALID_ARG
    del g
    # the context still computes (it was not poisoned)
    p = mils.periodogram(t, y, dy, c.f0, c.df, c.nf, ctx=ctx).cpu().numpy()
    ref = oracle.periodogram(c.t, c.y, c.dy, c.f0, c.df, nf=c.nf)
    assert np.max(np.abs(p - ref)) <= 1e-8 * np.max(np.abs(ref))
    # plan made with a smaller curve of the same frequency grid: the
    # workspace is too small for the larger one
    small = workloads.single_small(seed=1, nd=200, nf=c.nf)
    ctx2 = mils.Context(0)
    mils.periodogram(dev(small.t), dev(small.y), dev(small.dy), small.f0, small.df, small.nf,
                     ctx=ctx2)
    g, st = _capture(ctx2, c, t, y, dy, out)
    assert st == mils.MILS_ERR_BUSY
    del g
    p2 = mils.periodogram(t, y, dy, c.f0, c.df, c.nf, ctx=ctx2).cpu().numpy()
    assert np.max(np.abs(p2 - p)) <= 1e-13 * np.max(np.abs(p))
    ctx.close()
    ctx2.close()


def test_graph_survives_later_workspace_growth():
    """Capture a warm call, then grow the context's workspace with a larger
    uncaptured call; every replay of the graph still gives the eager result
    of the captured call."""
    c = workloads.single_small(seed=2, nd=500, nf=6000)
    big = workloads.single_large(seed=3, nd=60_000, span_years=2)
    t, y, dy = dev(c.t), dev(c.y), dev(c.dy)
    ctx = mils.Context(0)
    eager = mils.periodogram(t, y, dy, c.f0, c.df, c.nf, ctx=ctx).cpu().numpy()
    out = torch.empty(c.nf, dtype=torch.float64, device="cuda")
    g, st = _capture(ctx, c, t, y, dy, out)
    assert st == mils.MILS_OK
    pb = mils.periodogram(dev(big.t), dev(big.y), dev(big.dy), big.f0, big.df, big.nf,
                          ctx=ctx).cpu().numpy()
    assert np.isfinite(pb).all()
    for i in range(3):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        r = out.cpu().numpy()
        assert np.max(np.abs(r - eager)) <= 1e-13 * np.max(np.abs(eager)), i
    del g
    ctx.close()
