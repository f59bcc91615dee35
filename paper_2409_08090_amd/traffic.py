"""HBM traffic per kernel from two rocprofv3 counter runs.

Runs (from the repository root, on the GPU):

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir_fetch> -o run -- \\
        python3 bench.py --steps 3 --warmup 1 --no-cpu-baseline --no-extra \\
        --no-batch --no-serve --calibrate-copy
    rocprofv3 --pmc WRITE_SIZE  ... same with -d <dir_write>
    python3 -m paper_2409_08090_amd.traffic <dir_fetch> <dir_write> > traffic.json

FETCH_SIZE / WRITE_SIZE are read in KiB per dispatch.  Each is scaled by the
ratio between the bytes a plain device copy of known size moves (read once,
written once; bench.py --calibrate-copy runs one of 2^30 bytes) and what the
same counter reads for that copy.  Dispatches of the periodogram are named by
their stage; the two FFT pass launches of a step are told apart by order.
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
    ("k_stats", "stats"), ("k_lowfreq", "stats"), ("k_bins_sorted", "bin_sort"),
    ("k_sort", "bin_sort"), ("k_scan", "bin_sort"), ("k_spread", None),
    ("k_fft_pass", None), ("k_fft_last", "fft_last_power"),
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


def stage_bytes(disp, scale):
    """Average scaled bytes per launch of each stage of the last full step."""
    per = defaultdict(list)
    pass_idx = 0
    for _, name, kib in disp:
        stage = None
        if "k_spread" in name:
            stage = "spread_2f" if "Li2ELi1E" in name or "<double, 2, 1>" in name or \
                "<float, 2, 1>" in name else "spread_f"
        elif "k_fft_pass" in name:
            stage = f"fft_pass_{pass_idx}"
            pass_idx += 1
        elif "k_fft_last" in name:
            stage = "fft_last_power"
            pass_idx = 0
        else:
            for key, st in STAGE_OF:
                if key in name and st:
                    stage = st
                    break
        if stage:
            per[stage].append(kib * 1024.0 * scale)
    return {k: sum(v) / len(v) for k, v in per.items()}


def copy_scale(disp):
    cands = [kib for _, name, kib in disp if "copyBuffer" in name or "copy" in name.lower()]
    if not cands:
        return None
    kib = max(cands)
    return (COPY_BYTES / 1024.0) / kib if kib > 0 else None


def kernel_source_hash(root):
    h = hashlib.sha256()
    csrc = os.path.join(root, "paper_2409_08090_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        if fn.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(csrc, fn), "rb") as f:
                h.update(fn.encode())
                h.update(f.read())
    return h.hexdigest()[:16]


def main(argv):
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
