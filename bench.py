#!/usr/bin/env python3
"""Benchmark of the NUFFT Lomb-Scargle hot path on one MI355X.

A step is one whole periodogram of the single large light curve (N_d = 1e6
points over 3650 days with seasonal gaps, N_f = 1.2e7 frequencies, FP64,
eps = 1e-9): statistics, binning, both spreads, the three-pass FFT of the
three grids, deconvolution, crop and power.  Inputs are resident in HBM
before the timed region; the plan (twiddles, kernel transform) is cached from
the warm-up, as a NUFFT plan is.  Prints ONE JSON line.

Also reported (in "extra"): the FP32 precision form on the same curve, and the
error of both against the oracle on the sampled frequencies used for the CPU
baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "N_d·N_f-equiv sums/s FP64 vs FP32-batched at stated error; p50/p99 request latency"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nd", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-shared", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one device copy of 2^30 bytes (HBM counter calibration)")
    ap.add_argument("--serve-seconds", type=float, default=4.0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle sample")
    return ap.parse_args()


def active_fraction(t, df, geo, plan, tau):
    """Fraction of grid rows the spread writes (rows within half a kernel width
    of a point), from the host copy of t; used in the algorithmic byte model."""
    n = plan["n"]
    rows = plan["len"][0] if plan["npass"] > 1 else 1
    S1 = n // rows
    u = n * np.mod(geo * df * (t - tau), 1.0)
    hw = plan["width"] / 2 + 1
    active = np.zeros(rows, bool)
    for off in (-hw, 0.0, hw):
        active[(np.floor(np.mod(u + off, n) / S1)).astype(np.int64)] = True
    return active.mean()


def byte_model(c, plan, csize):
    """Algorithmic bytes per launch of each stage (see the design notes):
    inputs read once, spread writes of the active rows, every FFT pass reading
    and writing each grid once (the first pass reads only active rows), the
    last pass writing only the power and reading the kernel-transform table."""
    n, nd, nf = plan["n"], c.nd, c.nf
    tau = c.t.min()
    rf = active_fraction(c.t, c.df, 1, plan, tau)
    r2 = active_fraction(c.t, c.df, 2, plan, tau)
    ng = 3
    m = {
        "stats": 24.0 * nd,
        "lowfreq": 24.0 * nd,
        "bin_sort": 8.0 * nd + 4.0 * (n // plan["bin"] + 1),
        "spread_f": 24.0 * nd + 2 * rf * n * csize,
        "spread_2f": 16.0 * nd + r2 * n * csize,
        "fft_pass_0": (2 * rf + r2) * n * csize + ng * n * csize,
        "fft_pass_1": 2.0 * ng * n * csize,
        "fft_pass_2": 2.0 * ng * n * csize,
        "fft_last_power": ng * n * csize + 8.0 * nf + 8.0 * (nf // 2 + 1),
    }
    return m, rf, r2


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by frequency band across GPUs, see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2409_08090_amd import mils, traffic as trafficmod, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    c = workloads.single_large(seed=1, nd=args.nd)
    eps = 1e-9
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    t, y, dy = to(c.t), to(c.y), to(c.dy)
    power = torch.empty(c.nf, dtype=torch.float64, device=dev)
    ctx = mils.Context(0)
    stream = torch.cuda.current_stream()

    def step(prec="fp64", e=eps, out=power, sync=False):
        mils.periodogram(t, y, dy, c.f0, c.df, c.nf, eps=e, precision=prec, out=out,
                         stream=stream, ctx=ctx, sync=sync)

    for _ in range(max(1, args.warmup)):
        step(sync=True)
    torch.cuda.synchronize()
    plan = mils.plan_info(c.nd, c.nf, eps, "fp64", c.f0, c.df)
    bytes_model, rf, r2 = byte_model(c, plan, 16)
    # stage table: every stage timed with HIP events (outside the timed region:
    # the events of all stages slow a periodogram by ~6%)
    ctx.profile_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    stages = {}
    for name, (ms, n) in prof.items():
        per_step = ms / args.steps
        b = bytes_model.get(name, 0.0)
        stages[name] = {"ms_per_step": round(per_step, 5),
                        "launches_per_step": round(n / args.steps, 3), "alg_bytes": b,
                        "alg_GBs": round(b / (per_step * 1e-3) / 1e9, 1)}
    # The roofline's kernel: the costliest stage that is one kernel launch per
    # periodogram (a middle FFT pass or the last pass), so that its average
    # launch duration is what the kernel trace reports for it.
    single = [k for k in prof if prof[k][1] == args.steps and
              (k.startswith("fft_pass_") and k != "fft_pass_0" or k == "fft_last_power")]
    dom = max(single, key=lambda k: prof[k][0])
    # timed region: only the roofline kernel carries HIP events
    ctx.profile_enable(True, stages=[dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.check(mils.load().mils_context_status(ctx.handle))
    tprof = ctx.profile_read()
    ctx.profile_enable(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    sums = float(c.nd) * float(c.nf)
    value = sums / (ms_per_step * 1e-3)
    dom_ms = tprof[dom][0] / tprof[dom][1]
    achieved = bytes_model[dom] / (dom_ms * 1e-3) / 1e9
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic_single_large_fp64.json")
    if os.path.exists(tpath):
        try:
            rec = json.load(open(tpath))
            if rec.get("kernel_hash") == trafficmod.kernel_source_hash(ROOT) and \
                    dom in rec.get("bytes", {}):
                traffic = rec["bytes"][dom]
        except Exception:
            traffic = None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dom}
    whole_path_bytes = sum(bytes_model[k] for k in prof)
    extra = {"stages": stages, "active_rows": {"f": round(rf, 4), "2f": round(r2, 4)},
             "plan": plan, "whole_path_alg_GBs": round(whole_path_bytes / (ms_per_step * 1e-3) / 1e9, 1)}

    if args.calibrate_copy:
        src = torch.empty(trafficmod.COPY_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # FP32 precision form on the same curve
    if not args.no_extra:
        p32 = torch.empty_like(power)
        for _ in range(2):
            step("fp32", 1e-5, p32, sync=True)
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        for _ in range(args.steps):
            step("fp32", 1e-5, p32)
        torch.cuda.synchronize()
        a1 = time.perf_counter()
        ms32 = (a1 - a0) * 1e3 / args.steps
        extra["fp32_form"] = {"ms_per_step": round(ms32, 4), "value": sums / (ms32 * 1e-3),
                              "eps": 1e-5}

    # batched form: 10,000 series in one persistent launch, FP64 and FP32
    if not args.no_batch:
        curves = workloads.batch(seed=3)
        bt, by, bdy, nd_off, nf_off, f0s, dfs = mils.pack_curves(curves, device=dev)
        bout = torch.empty(int(nf_off[-1]), dtype=torch.float64, device=dev)
        bsums = float(sum(float(c.nd) * float(c.nf) for c in curves))
        extra["batch"] = {"ncurves": len(curves), "sum_nd_nf": bsums}
        for prec, e in (("fp64", 1e-9), ("fp32", 1e-5)):
            for _ in range(2):
                mils.periodogram_batch(bt, by, bdy, nd_off, nf_off, f0s, dfs, eps=e,
                                       precision=prec, out=bout, ctx=ctx, stream=stream)
            torch.cuda.synchronize()
            b0 = time.perf_counter()
            nb = max(3, args.steps // 4)
            for _ in range(nb):
                mils.periodogram_batch(bt, by, bdy, nd_off, nf_off, f0s, dfs, eps=e,
                                       precision=prec, out=bout, ctx=ctx, stream=stream)
            torch.cuda.synchronize()
            bms = (time.perf_counter() - b0) * 1e3 / nb
            extra["batch"][prec] = {"ms_per_batch": round(bms, 3),
                                    "value": bsums / (bms * 1e-3), "eps": e}

    # shared observation times: 8 series on the large curve's times, one dy
    # row for all (the weight-only sums run once), FP64 and FP32
    if not args.no_shared and not args.no_extra:
        sh = workloads.shared_times(seed=5, nd=c.nd, nseries=8)
        st_t, st_y, st_dy = to(sh.t), to(sh.y), to(sh.dy[0])
        sout = torch.empty((sh.nseries, sh.nf), dtype=torch.float64, device=dev)
        ssums = float(sh.nseries) * float(sh.nd) * float(sh.nf)
        extra["shared_times"] = {"nseries": sh.nseries, "nd": sh.nd, "nf": sh.nf}
        for prec, e in (("fp64", 1e-9), ("fp32", 1e-5)):
            for _ in range(2):
                mils.periodogram_shared_t(st_t, st_y, st_dy, sh.f0, sh.df, sh.nf, eps=e,
                                          precision=prec, out=sout, ctx=ctx, stream=stream)
            torch.cuda.synchronize()
            h0 = time.perf_counter()
            nrep = max(3, args.steps // 4)
            for _ in range(nrep):
                mils.periodogram_shared_t(st_t, st_y, st_dy, sh.f0, sh.df, sh.nf, eps=e,
                                          precision=prec, out=sout, ctx=ctx, stream=stream)
            torch.cuda.synchronize()
            hms = (time.perf_counter() - h0) * 1e3 / nrep
            extra["shared_times"][prec] = {"ms_per_call": round(hms, 3),
                                           "ms_per_series": round(hms / sh.nseries, 4),
                                           "value": ssums / (hms * 1e-3), "eps": e}
        del st_t, st_y, st_dy, sout

    # serving: open-loop Poisson arrivals at 2000 requests/s of mixed sizes and
    # precisions (a pool of 192 synthetic curves with N_d log-uniform in
    # [50, 2e5], reused by the arrivals), continuous batching on 3 lanes.  A
    # warm-up pass submits every pool curve once in each precision (the
    # server creates the plans of each size on first use); the latencies are
    # those of the timed window's requests (submit -> result in host memory),
    # with the warm-up's own (cold) latencies reported beside them.
    if not args.no_serve:
        rng = np.random.default_rng(4)
        pool = []
        for _ in range(192):
            ndq = int(np.floor(np.exp(rng.uniform(np.log(50), np.log(200_000)))))
            pool.append(workloads.batch_curve(rng, ndq))
        srv = mils.Server(0, lanes=3)

        def lat_ms(tickets):
            out = []
            for tk, nfq in tickets:
                srv.wait(tk)
                rcq, _, stq = srv.take(tk, nfq)
                if rcq == mils.MILS_OK:
                    out.append((stq["done_s"] - stq["submit_s"]) * 1e3)
            return np.array(out)

        warm = []
        for cq in pool:
            for prec, e in (("fp32", 1e-5), ("fp64", 1e-9)):
                rc, tk = srv.submit(cq.t, cq.y, cq.dy, cq.f0, cq.df, cq.nf, eps=e,
                                    precision=prec)
                if rc == mils.MILS_OK:
                    warm.append((tk, cq.nf))
        cold = lat_ms(warm)
        rate, dur = 2000.0, args.serve_seconds
        arrivals = np.cumsum(rng.exponential(1.0 / rate, int(rate * dur * 1.2)))
        arrivals = arrivals[arrivals < dur]
        picks = rng.integers(0, len(pool), arrivals.size)
        precs = rng.random(arrivals.size) < 0.5
        tickets = []
        busy = 0
        s0 = time.perf_counter()
        for a_t, pi, use32 in zip(arrivals, picks, precs):
            while time.perf_counter() - s0 < a_t:
                pass
            cq = pool[pi]
            prec, e = ("fp32", 1e-5) if use32 else ("fp64", 1e-9)
            rc, tk = srv.submit(cq.t, cq.y, cq.dy, cq.f0, cq.df, cq.nf, eps=e, precision=prec)
            if rc == mils.MILS_OK:
                tickets.append((tk, cq.nf))
            else:
                busy += 1
        lat = lat_ms(tickets)
        wall = time.perf_counter() - s0
        ss = srv.stats()
        lane_err = srv.last_error()
        srv.close()
        done_sums = float(sum(float(pool[pi].nd) * float(pool[pi].nf) for pi in picks))
        extra["serving"] = {"rate_req_s": rate, "seconds": dur, "offered": int(arrivals.size),
                            "completed": int(lat.size), "rejected": busy,
                            "p50_ms": round(float(np.percentile(lat, 50)), 3),
                            "p99_ms": round(float(np.percentile(lat, 99)), 3),
                            "max_ms": round(float(lat.max()), 3),
                            "sustained_sums_per_s": done_sums / wall,
                            "warmup": {"requests": int(cold.size),
                                       "p50_ms": round(float(np.percentile(cold, 50)), 3),
                                       "max_ms": round(float(cold.max()), 3)},
                            "mean_batch": round(ss["mean_batch"], 2), "batches": ss["batches"],
                            "peak_inflight_bytes": ss["peak_inflight_bytes"],
                            "failed": ss["failed"], "dead_lanes": ss["dead_lanes"]}
        if lane_err:
            extra["serving"]["lane_error"] = lane_err

    # the brute-force comparison (Sec. 2.1): every sum term by term in FP64 on
    # the first 1.2e6 frequencies of the same curve (last of the GPU legs: a
    # second of full FP64 load would slow what follows)
    if not args.no_extra:
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
        extra["direct_sum"] = {"nf": nfd, "seconds": round(dsec, 3), "value": dval,
                               "transform_speedup": round(value / dval, 1),
                               "transform_error_vs_direct": float(
                                   (power[:nfd] - pd).abs().max() / pd.abs().max())}
        del pd

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        rng = np.random.default_rng(2)
        # calibrate the sample size on a few frequencies, then time the sample
        oracle.periodogram(c.t, c.y, c.dy, c.f0, c.df, k=rng.integers(0, c.nf, 8))  # thread start-up
        k0 = rng.integers(0, c.nf, 64)
        s0 = time.perf_counter()
        oracle.periodogram(c.t, c.y, c.dy, c.f0, c.df, k=k0)
        per = (time.perf_counter() - s0) / k0.size
        nk = int(max(16, min(40000, args.cpu_seconds / max(per, 1e-6))))
        top = np.argsort(power.cpu().numpy())[-20:]
        ks = np.unique(np.concatenate([rng.integers(0, c.nf, nk), top]))
        s1 = time.perf_counter()
        ref = oracle.periodogram(c.t, c.y, c.dy, c.f0, c.df, k=ks)
        el = time.perf_counter() - s1
        cpu = {"value": float(c.nd) * ks.size / el, "unit": "sums/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"{ks.size} frequencies of the N_d=1e6, N_f=1.2e7 FP64 curve "
                         f"(random k plus the 20 strongest GPU peaks), {el:.1f} s"}
        p64 = power.cpu().numpy()
        extra["error_fp64"] = float(np.max(np.abs(p64[ks] - ref)) / np.max(np.abs(ref)))
        if "fp32_form" in extra:
            e32 = float(np.max(np.abs(p32.cpu().numpy()[ks] - ref)) / np.max(np.abs(ref)))
            extra["fp32_form"]["error_vs_oracle"] = e32

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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "single large light curve FP64: N_d=1e6 times over 3650 d with "
                               "120-day gaps, N_f=1.2e7, df=1/18250, eps=1e-9",
                   "nd": c.nd, "nf": c.nf, "eps": eps, "precision": "fp64"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
