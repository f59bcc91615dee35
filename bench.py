#!/usr/bin/env python3
"""Benchmark of the NUFFT Lomb-Scargle hot path on one MI355X.

A step is one whole periodogram of the single large light curve (N_d = 1e6
points over 3650 days with seasonal gaps, N_f = 1.2e7 frequencies, FP64,
eps = 1e-9): statistics, binning, both spreads, the FFT of the three grids,
deconvolution, crop and power.  Inputs are resident in HBM before the timed
region; the plan (twiddles, kernel transform) is cached from the warm-up, as
a NUFFT plan is, and repeated calls replay the context's captured graph.
Prints ONE JSON line.

roofline: the whole periodogram's algorithmic bytes (every input read once,
the power written once, the half table of the kernel transform, and per grid
v 2(1 + rho_v) n c: spread writes of the cells near a point, a first FFT pass
reading those and writing n c, a last pass reading n c) over ms_per_step,
against 8 TB/s; the dense model (4 n c per grid) beside it; and, as
roofline.kernel, the last FFT pass alone, timed with HIP events.

Also reported: the FP32 form, the small curve's call latency, the batched
form (10^4 curves) with its HBM and FFT-arithmetic fractions, shared
observation times, the serving loop on a fresh Poisson request stream, the
FP64 direct sums, and the CPU baselines (the oracle and a plain host FP64
NUFFT, built for and run on this host's cores); every GPU result form with
its error against the oracle on sampled frequencies.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "N_d·N_f-equiv sums/s FP64 vs FP32-batched at stated error; p50/p99 request latency"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6
EPS = {"fp64": 1e-9, "fp32": 1e-5}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nd", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-host-nufft", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="only the FP64 headline leg")
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-shared", action="store_true")
    ap.add_argument("--fp32", action="store_true",
                    help="headline leg in FP32 (eps 1e-5) instead of FP64 (profiling runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one device copy of 2^30 bytes (HBM counter calibration)")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="largest CPU time of the oracle sample")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_threads():
    env = os.environ.get("OMP_NUM_THREADS")
    n = len(os.sched_getaffinity(0))
    return min(n, int(env)) if env and env.isdigit() and int(env) > 0 else n


def covered_fraction(t, df, geo, n, w):
    """Fraction of the n grid cells within half a kernel width of a point of
    geometry geo (cells the spread writes), from the points' positions
    n * frac(geo df t) on the periodic grid: the union of width-w intervals."""
    u = np.sort(np.mod(geo * df * (t - t.min()), 1.0) * n)
    gaps = np.diff(np.concatenate([u, [u[0] + n]]))
    return float(min(n, np.minimum(gaps, w).sum())) / n


def byte_models(c, plan, csize):
    """(B_alg, dense, rho_f, rho_2f) for a periodogram of curve c on plan."""
    n, w = plan["n"], plan["width"]
    rf = covered_fraction(c.t, c.df, 1, n, w)
    r2 = covered_fraction(c.t, c.df, 2, n, w)
    io = 24.0 * c.nd + 8.0 * c.nf + 4.0 * c.nf
    b_alg = io + sum(2.0 * (1.0 + r) * n * csize for r in (rf, rf, r2))
    dense = io + 3 * 4.0 * n * csize
    return b_alg, dense, rf, r2


# the FFT passes bench.py times alone for roofline.kernel: the longer one is
# reported, with its algorithmic bytes
FFT_STAGES = ("fft_pass_0", "fft_last_power")


def kernel_bytes(stage, n, csize, rf, r2, nf):
    """Algorithmic bytes of one launch of an FFT pass over the three grids:
    the first pass reads the active rows (fractions rho) and writes every
    cell; the last pass reads every cell, one kernel-transform factor (4
    bytes: half the table) and writes one power per frequency."""
    if stage == "fft_pass_0":
        return (3.0 + 2.0 * rf + r2) * n * csize
    return 3.0 * n * csize + 12.0 * nf


def kernel_name(stage, plan, prec):
    if stage == "fft_pass_0":
        return "k_fft2_first" if plan["fft2"] else "k_fft_pass"
    if not plan["fft2"]:
        return "k_fft_last"
    return "k_fft2_last_seq" if prec == "fp32" else "k_fft2_last"


def peaks(p, m=3, sep=1000):
    """Indices of the m strongest peaks at least sep bins apart."""
    q = p.copy()
    out = []
    for _ in range(m):
        k = int(np.argmax(q))
        out.append(k)
        q[max(0, k - sep):k + sep + 1] = -np.inf
    return out


def subsample(nf, pk, rng, nrand):
    """The cfg2 frequency subsample: nrand uniform-random k, 1000 consecutive
    k around each peak, 1000 at each band edge."""
    ks = [rng.integers(0, nf, nrand), np.arange(1000), np.arange(nf - 1000, nf)]
    for k in pk:
        ks.append(np.arange(max(0, k - 500), min(nf, k + 500)))
    return np.unique(np.concatenate(ks))


def rel_err(p, ref):
    return float(np.max(np.abs(p - ref)) / np.max(np.abs(ref)))


def pct(a, q):
    return round(float(np.percentile(np.asarray(a), q)), 4)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path would shard by frequency band across GPUs; see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2409_08090_amd import mils, traffic as trafficmod, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    mils.load()  # fails loudly when the HIP library is not built
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)  # noqa: E731
    ctx = mils.Context(0)
    extra = {}

    # ------------------------------------------------------------ headline leg
    c = workloads.single_large(seed=1, nd=args.nd)
    prec = "fp32" if args.fp32 else "fp64"
    eps = EPS[prec]
    t, y, dy = to(c.t), to(c.y), to(c.dy)
    power = torch.empty(c.nf, dtype=torch.float64, device=dev)

    def step(pr=prec, out=power, sync=False):
        mils.periodogram(t, y, dy, c.f0, c.df, c.nf, eps=EPS[pr], precision=pr, out=out,
                         stream=stream, ctx=ctx, sync=sync)

    def timed(pr, out, nsteps):
        """Wall time per step over nsteps steps (graph replay, no events)."""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            step(pr, out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / nsteps
        ctx.check(mils.context_status(ctx))
        return ms

    def event_steps(pr, out, nsteps):
        """Device time of each step between two events on the call's stream."""
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(nsteps)]
        for a, b in ev:
            a.record(stream)
            step(pr, out)
            b.record(stream)
        torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in ev]

    def stage_table(pr, out, nsteps, models):
        """Per-stage HIP-event times (outside the timed region: the events
        switch graph replay off and cost a few percent)."""
        ctx.profile_enable(True)
        for _ in range(nsteps):
            step(pr, out)
        torch.cuda.synchronize()
        prof = ctx.profile_read()
        ctx.profile_enable(False)
        return {k: {"ms_per_step": round(ms / nsteps, 5),
                    "launches_per_step": round(nl / nsteps, 3)} for k, (ms, nl) in prof.items()}

    def kernel_time(pr, out, stage, nsteps):
        """Average duration of one stage's launch, the other stages untimed."""
        ctx.profile_enable(True, stages=[stage])
        for _ in range(nsteps):
            step(pr, out)
        torch.cuda.synchronize()
        ms, nl = ctx.profile_read()[stage]
        ctx.profile_enable(False)
        return ms / nl

    log(f"headline {prec}: warm-up")
    for _ in range(max(1, args.warmup)):
        step(sync=True)
    torch.cuda.synchronize()
    log("headline: timed region")
    ms_per_step = timed(prec, power, args.steps)
    sums = float(c.nd) * float(c.nf)
    value = sums / (ms_per_step * 1e-3)
    ev_ms = event_steps(prec, power, args.steps)
    plan = mils.plan_info(c.nd, c.nf, eps, prec, c.f0, c.df)
    csize = 8 if prec == "fp32" else 16
    b_alg, b_dense, rf, r2 = byte_models(c, plan, csize)
    stages = stage_table(prec, power, args.steps, None)
    # the dominant kernel: the longer of the two FFT passes, each timed alone
    k_times = {st: kernel_time(prec, power, st, args.steps) for st in FFT_STAGES}
    kname = max(k_times, key=k_times.get)
    k_ms = k_times[kname]
    k_bytes = kernel_bytes(kname, plan["n"], csize, rf, r2, c.nf)

    def stored_traffic(pr, stage):
        """(bytes per periodogram, bytes of the stage) from the counter runs
        kept in profiles/, or (None, None) when absent or taken on other
        kernel sources."""
        tpath = os.path.join(ROOT, "profiles", f"traffic_single_large_{pr}.json")
        try:
            rec = json.load(open(tpath))
            if rec.get("kernel_hash") == trafficmod.kernel_source_hash(ROOT):
                return float(sum(rec["bytes"].values())), rec["bytes"].get(stage)
        except (OSError, ValueError, KeyError):
            pass
        return None, None

    tr_total, tr_kernel = stored_traffic(prec, kname)
    achieved = b_alg / (ms_per_step * 1e-3) / 1e9
    roofline = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr_total,
        "scope": "whole periodogram per step: B_alg = 24 N_d + 12 N_f + sum over the 3 grids "
                 "of 2 (1 + rho_v) n c, over ms_per_step",
        "alg_bytes": b_alg, "rho": {"f": round(rf, 4), "2f": round(r2, 4)},
        "n": plan["n"], "c": csize,
        "dense_bytes": b_dense,
        "dense_frac": round(b_dense / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "traffic_vs_alg": round(tr_total / b_alg, 3) if tr_total else None,
        "kernel": {"name": kernel_name(kname, plan, prec),
                   "stage": kname, "avg_us": round(k_ms * 1e3, 2),
                   "other_pass_us": {st: round(v * 1e3, 2) for st, v in k_times.items()
                                     if st != kname},
                   "alg_bytes": k_bytes,
                   "achieved": round(k_bytes / (k_ms * 1e-3) / 1e9, 1),
                   "frac": round(k_bytes / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "traffic": tr_kernel},
    }
    extra["events_ms_per_step"] = {"median": pct(ev_ms, 50), "min": round(min(ev_ms), 4),
                                   "p90": pct(ev_ms, 90)}
    extra["stages"] = stages
    extra["plan"] = plan
    log(f"headline: {ms_per_step:.4f} ms/step, frac {roofline['frac']}")

    if args.calibrate_copy:
        src = torch.empty(trafficmod.COPY_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ------------------------------------------------------------ FP32 form
    p32 = None
    if not args.no_extra and not args.fp32:
        log("FP32 form")
        p32 = torch.empty_like(power)
        for _ in range(2):
            step("fp32", p32, sync=True)
        ms32 = timed("fp32", p32, args.steps)
        plan32 = mils.plan_info(c.nd, c.nf, EPS["fp32"], "fp32", c.f0, c.df)
        b32, d32, rf32, r232 = byte_models(c, plan32, 8)
        kt32 = {st: kernel_time("fp32", p32, st, args.steps) for st in FFT_STAGES}
        kn32 = max(kt32, key=kt32.get)
        k32 = kt32[kn32]
        kb32 = kernel_bytes(kn32, plan32["n"], 8, rf32, r232, c.nf)
        extra["fp32_form"] = {
            "ms_per_step": round(ms32, 5), "value": sums / (ms32 * 1e-3), "eps": EPS["fp32"],
            "alg_bytes": b32, "frac": round(b32 / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "dense_frac": round(d32 / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "plan": {k: plan32[k] for k in ("n", "len", "width", "fft2")},
            "traffic": stored_traffic("fp32", kn32)[0],
            "kernel": {"name": kernel_name(kn32, plan32, "fp32"), "stage": kn32,
                       "avg_us": round(k32 * 1e3, 2),
                       "frac": round(kb32 / (k32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
            "stages": stage_table("fp32", p32, args.steps, None)}
        step("fp32", p32, sync=True)

    # ------------------------------------------------------------ small-curve latency
    if not args.no_extra and not args.no_latency:
        log("small-curve latency")
        c0 = workloads.single_small(seed=0)
        t0d, y0d, dy0d = to(c0.t), to(c0.y), to(c0.dy)
        out0 = torch.empty(c0.nf, dtype=torch.float64, device=dev)
        ctx0 = mils.Context(0)
        lat = {}
        for graphs in (True, False):
            ctx0.set_graphs(graphs)
            samples = []
            for i in range(330):
                torch.cuda.synchronize()
                a = time.perf_counter()
                mils.periodogram(t0d, y0d, dy0d, c0.f0, c0.df, c0.nf, out=out0, stream=stream,
                                 ctx=ctx0)
                torch.cuda.synchronize()
                if i >= 30:
                    samples.append((time.perf_counter() - a) * 1e3)
            lat["graph_on" if graphs else "graph_off"] = {
                "median_ms": pct(samples, 50), "p99_ms": pct(samples, 99), "calls": len(samples)}
        ctx0.set_graphs(True)
        samples = []
        for i in range(330):
            a = time.perf_counter()
            td, yd, dyd = to(c0.t), to(c0.y), to(c0.dy)
            mils.periodogram(td, yd, dyd, c0.f0, c0.df, c0.nf, out=out0, stream=stream, ctx=ctx0)
            host = out0.cpu().numpy()
            if i >= 30:
                samples.append((time.perf_counter() - a) * 1e3)
        lat["host_to_host"] = {"median_ms": pct(samples, 50), "p99_ms": pct(samples, 99),
                               "calls": len(samples),
                               "note": "numpy inputs copied in, power copied out, graph on"}
        ref0 = None
        try:
            import oracle
            ref0 = oracle.periodogram(c0.t, c0.y, c0.dy, c0.f0, c0.df, nf=c0.nf)
            lat["error_vs_oracle"] = rel_err(host, ref0)
        except Exception as e:  # the oracle is test infrastructure; report, do not fail
            lat["error_vs_oracle"] = f"unavailable: {e}"
        lat["config"] = "N_d=1000 on [0,100], N_f=12000, f0=df=0.002, FP64, eps=1e-9"
        ctx0.close()
        extra["small_curve_latency"] = lat

    # ------------------------------------------------------------ batched form
    batch_sample = None
    if not args.no_extra and not args.no_batch:
        log("batched form")
        curves = workloads.batch(seed=3)
        bt, by, bdy, nd_off, nf_off, f0s, dfs = mils.pack_curves(curves, device=dev)
        bout = torch.empty(int(nf_off[-1]), dtype=torch.float64, device=dev)
        bsums = float(sum(float(q.nd) * float(q.nf) for q in curves))
        ex = {"ncurves": len(curves), "sum_nd_nf": bsums}
        rng = np.random.default_rng(6)
        pick = rng.choice(len(curves), 60, replace=False)
        batch_sample = (curves, pick, nf_off, {})
        for pr in ("fp64", "fp32"):
            e = EPS[pr]
            for _ in range(2):
                mils.periodogram_batch(bt, by, bdy, nd_off, nf_off, f0s, dfs, eps=e,
                                       precision=pr, out=bout, ctx=ctx, stream=stream)
            torch.cuda.synchronize()
            b0 = time.perf_counter()
            nb = max(5, args.steps // 4)
            for _ in range(nb):
                mils.periodogram_batch(bt, by, bdy, nd_off, nf_off, f0s, dfs, eps=e,
                                       precision=pr, out=bout, ctx=ctx, stream=stream)
            torch.cuda.synchronize()
            bms = (time.perf_counter() - b0) * 1e3 / nb
            ctx.check(mils.context_status(ctx))
            # staged byte model and FFT arithmetic (per curve: grid n = sigma nf,
            # the spread covering a fifth (f) and two fifths (2f) of the period
            # plus a kernel width; grids of at most 128 KiB stay in LDS)
            sig = 1.25 if pr == "fp64" else 1.5
            cs = 16 if pr == "fp64" else 8
            w = mils.plan_info(1000, 12000, e, pr)["width"]
            io = grid = flops = 0.0
            for q in curves:
                n = sig * q.nf
                io += 24.0 * q.nd + 12.0 * q.nf
                if n * cs > 128 * 1024:
                    for r in (0.2, 0.2, 0.4):
                        grid += 2.0 * (1.0 + min(1.0, r + w / n)) * n * cs
                flops += 3 * 5.0 * n * np.log2(n)
            b = io + grid
            peak_fl = (FP64_PEAK_TFLOPS if pr == "fp64" else FP32_PEAK_TFLOPS) * 1e12
            ex[pr] = {"ms_per_batch": round(bms, 3), "value": bsums / (bms * 1e-3), "eps": e,
                      "staged_bytes": b,
                      "hbm_frac": round(b / (bms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "fft_flops": flops,
                      "alu_frac": round(flops / (bms * 1e-3) / peak_fl, 4)}
            host = bout.cpu().numpy()
            batch_sample[3][pr] = {int(i): host[nf_off[i]:nf_off[i + 1]].copy() for i in pick}
        ex["fp32_vs_fp64_speedup"] = round(ex["fp64"]["ms_per_batch"] / ex["fp32"]["ms_per_batch"],
                                           3)
        ex["fp32_batched_vs_fp64_single_sums_per_s"] = round(ex["fp32"]["value"] / value, 4)
        extra["batch"] = ex
        del bt, by, bdy, bout

    # ------------------------------------------------------------ shared observation times
    shared_sample = None
    if not args.no_shared and not args.no_extra:
        log("shared observation times")
        sh = workloads.shared_times(seed=5, nd=c.nd, nseries=8)
        st_t, st_y, st_dy = to(sh.t), to(sh.y), to(sh.dy[0])
        sout = torch.empty((sh.nseries, sh.nf), dtype=torch.float64, device=dev)
        ssums = float(sh.nseries) * float(sh.nd) * float(sh.nf)
        ex = {"nseries": sh.nseries, "nd": sh.nd, "nf": sh.nf}
        shared_sample = (sh, {})
        for pr in ("fp64", "fp32"):
            e = EPS[pr]
            for _ in range(2):
                mils.periodogram_shared_t(st_t, st_y, st_dy, sh.f0, sh.df, sh.nf, eps=e,
                                          precision=pr, out=sout, ctx=ctx, stream=stream)
            torch.cuda.synchronize()
            h0 = time.perf_counter()
            nrep = max(3, args.steps // 4)
            for _ in range(nrep):
                mils.periodogram_shared_t(st_t, st_y, st_dy, sh.f0, sh.df, sh.nf, eps=e,
                                          precision=pr, out=sout, ctx=ctx, stream=stream)
            torch.cuda.synchronize()
            hms = (time.perf_counter() - h0) * 1e3 / nrep
            ctx.check(mils.context_status(ctx))
            ex[pr] = {"ms_per_call": round(hms, 3), "ms_per_series": round(hms / sh.nseries, 4),
                      "value": ssums / (hms * 1e-3), "eps": e}
            rng = np.random.default_rng(7)
            ks = np.unique(np.concatenate([rng.integers(0, sh.nf, 40), np.arange(8)]))
            shared_sample[1][pr] = (ks, sout[:, torch.from_numpy(ks).to(dev)].cpu().numpy())
        extra["shared_times"] = ex
        del st_t, st_y, st_dy, sout

    # ------------------------------------------------------------ serving
    serve_sample = None
    if not args.no_serve and not args.no_extra:
        serve_sample = serve_leg(args, mils, workloads, extra)

    # ------------------------------------------------------------ direct sums (Sec. 2.1)
    if not args.no_extra:
        log("direct sums")
        nfd = min(c.nf, 1_200_000)
        pd = torch.empty(nfd, dtype=torch.float64, device=dev)
        mils.direct_periodogram(t, y, dy, c.f0, c.df, 4096, out=pd[:4096], ctx=ctx,
                                stream=stream)
        torch.cuda.synchronize()
        d0 = time.perf_counter()
        mils.direct_periodogram(t, y, dy, c.f0, c.df, nfd, out=pd, ctx=ctx, stream=stream)
        torch.cuda.synchronize()
        dsec = time.perf_counter() - d0
        dval = float(c.nd) * nfd / dsec
        step(sync=True)
        extra["direct_sum"] = {"nf": nfd, "seconds": round(dsec, 3), "value": dval,
                               "transform_speedup": round(value / dval, 1),
                               "transform_error_vs_direct": float(
                                   (power[:nfd] - pd).abs().max() / pd.abs().max())}
        del pd

    # ------------------------------------------------------------ CPU baselines
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_leg(args, c, power, p32, prec, value, extra, batch_sample, shared_sample,
                      serve_sample)

    ctx.close()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "sums/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": "single large light curve: N_d=1e6 times over 3650 d with "
                               "120-day gaps, N_f=1.2e7, df=1/18250, "
                               + ("FP32 form eps=1e-5" if args.fp32 else "FP64 eps=1e-9"),
                   "nd": c.nd, "nf": c.nf, "eps": eps, "precision": prec},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


def serve_leg(args, mils, workloads, extra):
    """cfg4: open-loop Poisson arrivals of fresh requests (N_d log-uniform in
    [50, 2e5], N_f = 12 N_d, FP32 eps 1e-5 or FP64 eps 1e-9 by a fair coin).
    The server's plan classes are built first (mils_server_warm, timed), then
    one second of other fresh requests settles the lanes' buffers, then the
    timed window.  Latency is submit -> result in host memory."""
    log("serving: generating requests")
    nreq = int(round(args.serve_rate * args.serve_seconds))
    g0 = time.perf_counter()
    reqs = workloads.serving_requests(seed=4, nreq=nreq, rate=args.serve_rate)
    pre = workloads.serving_requests(seed=40, nreq=int(args.serve_rate), rate=args.serve_rate)
    gen_s = time.perf_counter() - g0
    srv = mils.Server(0, lanes=3)
    w0 = time.perf_counter()
    for pr in ("fp32", "fp64"):
        rc = srv.warm(12 * 200_000, eps=EPS[pr], precision=pr)
        if rc != mils.MILS_OK:
            raise RuntimeError(f"server warm-up failed: {rc} {srv.last_error()}")
    warm_s = time.perf_counter() - w0
    s_warm = srv.stats()
    sample_ix = set(range(0, nreq, max(1, nreq // 100)))
    kept = {}

    def run(stream_reqs, keep):
        tickets = []
        done = []
        stop = threading.Event()

        def consumer():
            i = 0
            while True:
                if i >= len(tickets):
                    if stop.is_set() and i >= len(tickets):
                        return
                    time.sleep(0.0005)
                    continue
                idx, tk, nfq = tickets[i]
                i += 1
                if srv.wait(tk, 120_000_000) != mils.MILS_OK:
                    done.append((idx, mils.MILS_ERR_TIMEOUT, 0.0, 0, 0.0, 0.0))
                    continue
                rcq, pq, stq = srv.take(tk, nfq)
                done.append((idx, rcq, stq["done_s"] - stq["submit_s"], stq["batch_size"],
                             stq["done_s"], stq["submit_s"]))
                if keep and idx in sample_ix and rcq == mils.MILS_OK:
                    kept[idx] = pq

        th = threading.Thread(target=consumer)
        th.start()
        busy = 0
        s0 = time.perf_counter()
        for idx, (a_t, cq, pr) in enumerate(stream_reqs):
            while True:
                dt = a_t - (time.perf_counter() - s0)
                if dt <= 0:
                    break
                if dt > 0.0008:
                    time.sleep(dt - 0.0005)
            rc, tk = srv.submit(cq.t, cq.y, cq.dy, cq.f0, cq.df, cq.nf, eps=EPS[pr],
                                precision=pr)
            if rc == mils.MILS_OK:
                tickets.append((idx, tk, cq.nf))
            else:
                busy += 1
        stop.set()
        th.join()
        return done, busy, time.perf_counter() - s0

    log("serving: settling run")
    st_pre = srv.stats()
    done_pre, _, _ = run(pre, False)
    s_pre = srv.stats()
    log("serving: timed window")
    done, busy, wall = run(reqs, True)
    s_end = srv.stats()
    lane_err = srv.last_error()
    srv.close()
    ok = [d for d in done if d[1] == mils.MILS_OK]
    lat = np.array([d[2] for d in ok]) * 1e3
    first = min(d[5] for d in ok)
    last = max(d[4] for d in ok)
    sums_done = float(sum(float(reqs[d[0]][1].nd) * float(reqs[d[0]][1].nf) for d in ok))
    ex = {"rate_req_s": args.serve_rate, "seconds": args.serve_seconds, "offered": nreq,
          "completed": len(ok), "failed": len(done) - len(ok), "rejected": busy,
          "fresh_requests": True,
          "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "max_ms": round(float(lat.max()), 3),
          "sustained_sums_per_s": sums_done / (last - first),
          "offered_sums_per_s": float(sum(float(q.nd) * float(q.nf) for _, q, _ in reqs))
          / args.serve_seconds,
          "wall_s": round(wall, 3),
          "mean_batch": round(float(np.mean([d[3] for d in ok])), 2),
          "plans_built_in_window": int(s_end["plans_built"] - s_pre["plans_built"]),
          "plan_build_ms_in_window": round(s_end["plan_build_ms"] - s_pre["plan_build_ms"], 3),
          "warm": {"seconds": round(warm_s, 3), "plans_built": int(s_warm["plans_built"]),
                   "plan_build_ms": round(s_warm["plan_build_ms"], 1)},
          "settling_run": {"requests": len(done_pre),
                           "plans_built": int(s_pre["plans_built"] - st_pre["plans_built"]),
                           "p50_ms": pct([d[2] * 1e3 for d in done_pre], 50),
                           "p99_ms": pct([d[2] * 1e3 for d in done_pre], 99)},
          "request_generation_s": round(gen_s, 1),
          "peak_inflight_bytes": s_end["peak_inflight_bytes"], "dead_lanes": s_end["dead_lanes"]}
    if lane_err:
        ex["lane_error"] = lane_err
    extra["serving"] = ex
    return reqs, kept


def cpu_leg(args, c, power, p32, prec, value, extra, batch_sample, shared_sample, serve_sample):
    """The oracle (built -O3 -march=native here) on the cfg2 frequency
    subsample of the large curve, timed; the GPU results' errors against it;
    the plain host FP64 NUFFT timed in full on the small curve, the large
    curve and the 10^4-curve batch."""
    import oracle
    log("CPU: building the oracle for this host")
    oracle.use_native()
    threads = oracle.num_threads()
    pw = power.cpu().numpy()
    rng = np.random.default_rng(2)
    oracle.periodogram(c.t, c.y, c.dy, c.f0, c.df, k=rng.integers(0, c.nf, 8))
    k0 = rng.integers(0, c.nf, 64)
    s0 = time.perf_counter()
    oracle.periodogram(c.t, c.y, c.dy, c.f0, c.df, k=k0)
    per = (time.perf_counter() - s0) / k0.size
    nrand = int(max(200, min(5000, (args.cpu_seconds / max(per, 1e-9)) - 5000)))
    ks = subsample(c.nf, peaks(pw), rng, nrand)
    log(f"CPU: oracle on {ks.size} frequencies (~{per * ks.size:.0f} s)")
    s1 = time.perf_counter()
    ref = oracle.periodogram(c.t, c.y, c.dy, c.f0, c.df, k=ks)
    el = time.perf_counter() - s1
    cpu = {"value": float(c.nd) * ks.size / el, "unit": "sums/s", "cores": threads,
           "kind": "oracle",
           "sample": f"{ks.size} frequencies of the N_d=1e6, N_f=1.2e7 curve ({nrand} uniform-"
                     "random k, 1000 around each of the 3 strongest peaks, 1000 at each band "
                     f"edge), every sum in FP64 with compensation, {el:.1f} s",
           "build": "gcc -O3 -march=native -fno-fast-math -ffp-contract=off, OpenMP"}
    extra[f"error_{prec}_vs_oracle"] = rel_err(pw[ks], ref)
    if p32 is not None:
        extra["fp32_form"]["error_vs_oracle"] = rel_err(p32.cpu().numpy()[ks], ref)
    # batched, shared-times and served results against the oracle on samples
    if batch_sample is not None:
        curves, pick, nf_off, res = batch_sample
        r = np.random.default_rng(8)
        errs = {pr: 0.0 for pr in res}
        for i in pick:
            q = curves[i]
            kq = np.unique(np.concatenate([r.integers(0, q.nf, 48), np.arange(8),
                                           [int(np.argmax(res["fp64"][int(i)]))]]))
            rq = oracle.periodogram(q.t, q.y, q.dy, q.f0, q.df, k=kq)
            for pr in res:
                errs[pr] = max(errs[pr], rel_err(res[pr][int(i)][kq], rq))
        for pr in errs:
            extra["batch"][pr]["error_vs_oracle"] = errs[pr]
        extra["batch"]["error_sample"] = f"{len(pick)} curves x ~57 frequencies"
    if shared_sample is not None:
        sh, res = shared_sample
        for pr, (ksh, vals) in res.items():
            e = 0.0
            for i in range(sh.nseries):
                rq = oracle.periodogram(sh.t, sh.y[i], sh.dy[i], sh.f0, sh.df, k=ksh)
                e = max(e, rel_err(vals[i], rq))
            extra["shared_times"][pr]["error_vs_oracle"] = e
    if serve_sample is not None:
        reqs, kept = serve_sample
        r = np.random.default_rng(9)
        errs = {}
        for idx, pq in kept.items():
            _, q, pr = reqs[idx]
            kq = np.unique(np.concatenate([r.integers(0, q.nf, 48), [int(np.argmax(pq))]]))
            rq = oracle.periodogram(q.t, q.y, q.dy, q.f0, q.df, k=kq)
            errs[pr] = max(errs.get(pr, 0.0), rel_err(pq[kq], rq))
        extra["serving"]["error_vs_oracle"] = errs
        extra["serving"]["error_sample"] = f"{len(kept)} requests x ~49 frequencies"
    if not args.no_host_nufft:
        cpu["host_nufft"] = host_nufft_leg(c, value, extra)
    return cpu


def host_nufft_leg(c, gpu_value, extra):
    """The plain host FP64 NUFFT (hostnufft/, -O3 -march=native, OpenMP on
    every host core of this process), timed in full."""
    import hostnufft
    from paper_2409_08090_amd import workloads
    log("CPU: host NUFFT")
    hostnufft.build(native=True)
    th = host_threads()
    out = {"cores": th, "build": "g++ -O3 -march=native, OpenMP", "kind": "plain host FP64 NUFFT"}
    c0 = workloads.single_small(seed=0)
    hostnufft.periodogram(c0.t, c0.y, c0.dy, c0.f0, c0.df, c0.nf, threads=th, native=True)
    ts = []
    for _ in range(3):
        a = time.perf_counter()
        hostnufft.periodogram(c0.t, c0.y, c0.dy, c0.f0, c0.df, c0.nf, threads=th, native=True)
        ts.append(time.perf_counter() - a)
    out["small_curve"] = {"ms": round(float(np.median(ts)) * 1e3, 3),
                          "value": c0.nd * c0.nf / float(np.median(ts)), "runs": 3}
    a = time.perf_counter()
    hostnufft.periodogram(c.t, c.y, c.dy, c.f0, c.df, c.nf, threads=th, native=True)
    s1 = time.perf_counter() - a
    out["large_curve"] = {"seconds": round(s1, 3), "value": c.nd * c.nf / s1, "runs": 1,
                          "gpu_speedup": round(gpu_value / (c.nd * c.nf / s1), 1)}
    curves = workloads.batch(seed=3)
    a = time.perf_counter()
    hostnufft.batch(curves, threads=th, native=True)
    s3 = time.perf_counter() - a
    bsums = float(sum(float(q.nd) * float(q.nf) for q in curves))
    out["batch"] = {"seconds": round(s3, 3), "value": bsums / s3, "runs": 1}
    if "batch" in extra and "fp32" in extra["batch"]:
        out["batch"]["gpu_fp32_speedup"] = round(extra["batch"]["fp32"]["value"] / (bsums / s3), 1)
    return out


if __name__ == "__main__":
    main()
