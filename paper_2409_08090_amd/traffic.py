"""HBM traffic per kernel from two rocprofv3 counter runs.

Runs (from the repository root, on the GPU):

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir_fetch> -o run -- \\
        python3 bench.py --steps 3 --warmup 1 --no-cpu-baseline --no-extra \\
        --no-batch --no-serve --calibrate-copy
    rocprofv3 --pmc WRITE_SIZE  ... same with -d <dir_write>
    python3 -m paper_2409_08090_amd.traffic <dir_fetch> <dir_write> > traffic.json

and, for SQ_ counter runs (at most 8 SQ_ counters per run),

    python3 -m paper_2409_08090_amd.traffic counters <dir> [<dir> ...] > counters.json

FETCH_SIZE / WRITE_SIZE are read in KiB per dispatch.  Each is scaled by the
ratio between the bytes a plain device copy of known size moves (read once,
written once; bench.py --calibrate-copy runs one of 2^30 bytes) and what the
same counter reads for that copy.  Dispatches of the periodogram are named by
their stage and summed per periodogram (the first FFT pass is two launches).
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

COPY_BYTES = 1 << 30
STAGE_OF = [
    ("k_stats", "stats"), ("k_lowfreq", "lowfreq"), ("k_bins_sorted", "bin_sort"),
    ("k_sort", "bin_sort"), ("k_scan", "bin_sort"), ("k_row_flags", "row_class"),
    ("k_row_compact", "row_class"),
    ("k_fft_last", "fft_last_power"), ("k_fft2_first", "fft_pass_0"),
    ("k_fft2_last", "fft_last_power"), ("k_fft2_out", "fft_out"),
]


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection*.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection csv under {d}")
    out = []
    for f in files:
        with open(f) as fh:
            out += list(csv.DictReader(fh))
    return out


def per_dispatch(d, counter):
    """[(dispatch_id, kernel_name, KiB)] in dispatch order."""
    acc = defaultdict(float)
    names = {}
    for r in _rows(d):
        if r.get("Counter_Name", "").strip() != counter:
            continue
        did = int(r["Dispatch_Id"])
        acc[did] += float(r["Counter_Value"])
        names[did] = r["Kernel_Name"]
    return [(k, names[k], acc[k]) for k in sorted(acc)]


def _is_2f(name):
    """The 2f-geometry spread (template arguments <Real, 2, 1, ...>)."""
    return "Li2ELi1E" in name or "<double, 2, 1" in name or "<float, 2, 1" in name


def stage_bytes(disp, scale):
    """Average scaled bytes per periodogram of each stage, over the complete
    periodograms in the trace (each starts with k_stats).  A multi-pass plan
    launches the first FFT pass twice (the 2f grid, then the two f grids,
    after the 2f spread): those two make stage fft_pass_0, and the i-th
    later pass launch is fft_pass_i.  A two-pass register-tile plan has one
    first-pass launch (fft_pass_0), its last pass and the transpose
    (fft_out).  The row classes of both geometries make stage row_class."""
    steps = []
    cur = None
    npass = 0
    fork = False
    for _, name, kib in disp:
        if "k_stats" in name and "k_stats_final" not in name:
            cur = defaultdict(float)
            steps.append(cur)
            npass = 0
            fork = False
        if cur is None:
            continue
        stage = None
        if "k_spread" in name:
            fork = fork or _is_2f(name)
            stage = "spread_2f" if _is_2f(name) else "spread_f"
        elif "k_fft_pass" in name:
            stage = f"fft_pass_{max(0, npass - 1) if fork else npass}"
            npass += 1
        else:
            for key, st in STAGE_OF:
                if key in name:
                    stage = st
                    break
        if stage:
            cur[stage] += kib * 1024.0 * scale
    done = [st for st in steps if "fft_last_power" in st]
    if not done:
        return {}
    keys = set().union(*done)
    return {k: sum(st.get(k, 0.0) for st in done) / len(done) for k in keys}


def copy_scale(disp):
    cands = [kib for _, name, kib in disp if "copyBuffer" in name or "copy" in name.lower()]
    if not cands:
        return None
    kib = max(cands)
    return (COPY_BYTES / 1024.0) / kib if kib > 0 else None


# The sources the single-series kernels are compiled from, and the planner
# that fixes their launch shapes: a change to any of them makes stored
# counter readings stale.
SINGLE_PATH_SOURCES = ("device_math.h", "fft2.h", "fft2_index.h", "fft_core.h", "kernels.h",
                       "kernels.hip", "mils_internal.h", "path_device.h", "plan.cpp", "plan.h")


def kernel_source_hash(root):
    h = hashlib.sha256()
    csrc = os.path.join(root, "paper_2409_08090_amd", "csrc")
    for fn in SINGLE_PATH_SOURCES:
        with open(os.path.join(csrc, fn), "rb") as f:
            h.update(fn.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name):
    """Kernel name without namespace, parameter list and the 'void ' prefix."""
    n = name.strip('"').replace("(anonymous namespace)::", "")
    if n.startswith("void "):
        n = n[5:]
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            n = n[:i]
            break
    return n.replace("mils::", "")


def kernel_counters(dirs, cycles_per_ns=2.4, num_cu=256):
    """Per kernel: dispatches, mean duration (ns) and the mean of every SQ_
    counter per dispatch, over one or more rocprofv3 --pmc runs of the same
    program; plus ratios that do not depend on the counters' units:
    valu_busy = SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES, lds_wait =
    SQ_WAIT_INST_LDS / SQ_WAVE_CYCLES, any_wait = SQ_WAIT_ANY / SQ_WAVE_CYCLES,
    bank_conflict = SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE, lds_util =
    SQ_LDS_IDX_ACTIVE / (num_cu * duration cycles) (the share of the CUs' LDS
    cycles spent on indexed accesses, against a peak of one access per CU
    and cycle), and instructions per wave."""
    acc = defaultdict(lambda: defaultdict(float))
    cnt = defaultdict(lambda: defaultdict(int))
    dur = defaultdict(list)
    for d in dirs:
        seen = set()
        for r in _rows(d):
            k = short_name(r["Kernel_Name"])
            c = r["Counter_Name"].strip()
            acc[k][c] += float(r["Counter_Value"])
            key = (r["Dispatch_Id"], c)
            if key not in seen:
                seen.add(key)
                cnt[k][c] += 1
            if (r["Dispatch_Id"], "dur") not in seen:
                seen.add((r["Dispatch_Id"], "dur"))
                dur[k].append(float(r["End_Timestamp"]) - float(r["Start_Timestamp"]))
    out = {}
    for k in acc:
        m = {c: acc[k][c] / cnt[k][c] for c in acc[k]}
        e = {"dispatches": max(cnt[k].values()), "mean_ns": sum(dur[k]) / len(dur[k])}
        e.update(m)
        wc = m.get("SQ_WAVE_CYCLES")
        if wc:
            for name, c in (("valu_busy", "SQ_ACTIVE_INST_VALU"), ("lds_wait", "SQ_WAIT_INST_LDS"),
                            ("any_wait", "SQ_WAIT_ANY"), ("lds_busy", "SQ_ACTIVE_INST_LDS")):
                if c in m:
                    e[name] = m[c] / wc
        if m.get("SQ_LDS_IDX_ACTIVE"):
            if "SQ_LDS_BANK_CONFLICT" in m:
                e["bank_conflict"] = m["SQ_LDS_BANK_CONFLICT"] / m["SQ_LDS_IDX_ACTIVE"]
            e["lds_util"] = m["SQ_LDS_IDX_ACTIVE"] / (num_cu * e["mean_ns"] * cycles_per_ns)
        if m.get("SQ_WAVES"):
            for name, c in (("valu_per_wave", "SQ_INSTS_VALU"), ("lds_per_wave", "SQ_INSTS_LDS"),
                            ("vmem_rd_per_wave", "SQ_INSTS_VMEM_RD")):
                if c in m:
                    e[name] = m[c] / m["SQ_WAVES"]
        out[k] = e
    return out


def main(argv):
    if len(argv) > 1 and argv[1] == "counters":
        json.dump(kernel_counters(argv[2:]), sys.stdout, indent=1)
        print()
        return
    dfetch, dwrite = argv[1], argv[2]
    fetch = per_dispatch(dfetch, "FETCH_SIZE")
    write = per_dispatch(dwrite, "WRITE_SIZE")
    sf, sw = copy_scale(fetch), copy_scale(write)
    fb = stage_bytes([x for x in fetch if "copy" not in x[1].lower()], sf or 1.0)
    wb = stage_bytes([x for x in write if "copy" not in x[1].lower()], sw or 1.0)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = {"kernel_hash": kernel_source_hash(root),
           "copy_scale": {"fetch": sf, "write": sw},
           "fetch_bytes": fb, "write_bytes": wb,
           "bytes": {k: fb.get(k, 0.0) + wb.get(k, 0.0) for k in set(fb) | set(wb)}}
    json.dump(out, sys.stdout, indent=1)
    print()


if __name__ == "__main__":
    main(sys.argv)
