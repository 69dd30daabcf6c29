"""Summaries of rocprofv3 output for the fused step kernel.

``python -m paper_1008_5113_amd.profiling summarize --trace DIR --fetch DIR --write DIR
--copy-fetch DIR --copy-write DIR --out-json FILE`` reads the CSV files that
``rocprofv3 --kernel-trace --stats`` and ``rocprofv3 --pmc FETCH_SIZE`` /
``--pmc WRITE_SIZE`` wrote (for bench.py and for bench.py --copy-calibration),
scales the counters by what they read for a plain 1 GiB device copy, and writes
the per-launch figures of the timed k_run dispatch to a JSON file.  The JSON
records a hash of the kernel sources; bench.py reports the traffic only while
the sources still hash the same.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(os.path.basename(p).encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def _rows(d, suffix):
    fs = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not fs:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    with open(fs[0]) as f:
        return list(csv.DictReader(f))


def _largest_dispatch(rows, name_part, prec=None):
    best = None
    for r in rows:
        if name_part not in r["Kernel_Name"]:
            continue
        if prec is not None and f"<{prec}>" not in r["Kernel_Name"]:
            continue
        dur = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        if best is None or dur > best[0]:
            best = (dur, r)
    return best


def summarize(trace, fetch, write, copy_fetch, copy_write, prec):
    cf = _largest_dispatch(_rows(copy_fetch, "counter_collection.csv"), "copyBuffer")[1]
    cw = _largest_dispatch(_rows(copy_write, "counter_collection.csv"), "copyBuffer")[1]
    fetch_scale = COPY_BYTES / (float(cf["Counter_Value"]) * 1024.0)
    write_scale = COPY_BYTES / (float(cw["Counter_Value"]) * 1024.0)
    f = _largest_dispatch(_rows(fetch, "counter_collection.csv"), "k_run", prec)[1]
    w = _largest_dispatch(_rows(write, "counter_collection.csv"), "k_run", prec)[1]
    stats = _rows(trace, "kernel_stats.csv")
    trace_rows = _rows(trace, "kernel_trace.csv")
    tr = _largest_dispatch(trace_rows, "k_run", prec)
    out = {
        "kernel": f"k_run<{prec}>",
        "source_hash": kernel_source_hash(),
        "fetch_kib": float(f["Counter_Value"]),
        "write_kib": float(w["Counter_Value"]),
        "fetch_scale": fetch_scale,
        "write_scale": write_scale,
        "hbm_bytes": float(f["Counter_Value"]) * 1024.0 * fetch_scale
        + float(w["Counter_Value"]) * 1024.0 * write_scale,
        "counter_dispatch_ms": (int(f["End_Timestamp"]) - int(f["Start_Timestamp"])) / 1e6,
        "trace_dispatch_ms": tr[0] / 1e6 if tr else None,
        "vgpr": int(f["VGPR_Count"]),
        "scratch": int(f["Scratch_Size"]),
        "grid": int(f["Grid_Size"]),
        "kernel_stats": [{k: s[k] for k in ("Name", "Calls", "AverageNs", "Percentage")} for s in stats[:8]],
    }
    return out


def main():
    ap = argparse.ArgumentParser()
    sp = ap.add_subparsers(dest="cmd")
    s = sp.add_parser("summarize")
    for k in ("trace", "fetch", "write", "copy_fetch", "copy_write"):
        s.add_argument("--" + k.replace("_", "-"), required=True)
    s.add_argument("--prec", type=int, default=1)
    s.add_argument("--out-json", required=True)
    args = ap.parse_args()
    if args.cmd != "summarize":
        ap.error("summarize is the only command")
    out = summarize(args.trace, args.fetch, args.write, args.copy_fetch, args.copy_write, args.prec)
    with open(args.out_json, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
