"""Summaries of rocprofv3 output for the fused step kernel and the per-phase
micro-benchmarks.

``python -m paper_1008_5113_amd.profiling summarize --trace DIR --fetch DIR --write DIR
--copy-fetch DIR --copy-write DIR --out-json FILE`` reads the CSV files that
``rocprofv3 --kernel-trace --stats`` and ``rocprofv3 --pmc FETCH_SIZE`` /
``--pmc WRITE_SIZE`` wrote (for bench.py and for bench.py --copy-calibration),
scales the counters by what they read for a plain 1 GiB device copy, and writes
the per-launch figures of the step kernel (every launch covers the same number
of steps) to a JSON file, with the launch configuration it was taken at.  The JSON
records a hash of the kernel sources; bench.py reports the traffic only while
the sources still hash the same.

``python -m paper_1008_5113_amd.profiling phases --trace DIR --fetch DIR --write DIR
--copy-fetch DIR --copy-write DIR --bench-log FILE --out-md FILE`` does the same
for ``bench.py --phases`` runs: per phase, the traced duration, algorithmic and
HBM bytes, and both rates against the 8 TB/s peak.
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
    """Hash of the sources the step kernel is compiled from (its translation
    unit: vmcdet.hip and the vmc_*.hpp headers it includes)."""
    h = hashlib.sha256()
    files = [os.path.join(HERE, "csrc", "vmcdet.hip")] + glob.glob(os.path.join(HERE, "csrc", "vmc_*.hpp"))
    for p in sorted(files):
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


def _dispatches(rows, name_part, prec=None):
    out = []
    for r in rows:
        if name_part not in r["Kernel_Name"]:
            continue
        if prec is not None and f"<{prec}>" not in r["Kernel_Name"]:
            continue
        out.append(r)
    return out


def summarize(trace, fetch, write, copy_fetch, copy_write, prec, launch):
    cf = _largest_dispatch(_rows(copy_fetch, "counter_collection.csv"), "copyBuffer")[1]
    cw = _largest_dispatch(_rows(copy_write, "counter_collection.csv"), "copyBuffer")[1]
    fetch_scale = COPY_BYTES / (float(cf["Counter_Value"]) * 1024.0)
    write_scale = COPY_BYTES / (float(cw["Counter_Value"]) * 1024.0)
    # every launch of the step kernel covers the same number of steps, so the
    # per-launch figure is the mean over its dispatches
    fr = _dispatches(_rows(fetch, "counter_collection.csv"), "k_run", prec)
    wr = _dispatches(_rows(write, "counter_collection.csv"), "k_run", prec)
    fetch_kib = sum(float(r["Counter_Value"]) for r in fr) / len(fr)
    write_kib = sum(float(r["Counter_Value"]) for r in wr) / len(wr)
    tr = _dispatches(_rows(trace, "kernel_trace.csv"), "k_run", prec)
    durs = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in tr]
    stats = _rows(trace, "kernel_stats.csv")
    return {
        "kernel": f"k_run<{prec}>",
        "source_hash": kernel_source_hash(),
        "launch": launch,
        "dispatches": {"trace": len(tr), "fetch": len(fr), "write": len(wr)},
        "fetch_kib_per_launch": fetch_kib,
        "write_kib_per_launch": write_kib,
        "fetch_scale": fetch_scale,
        "write_scale": write_scale,
        "hbm_bytes_per_launch": fetch_kib * 1024.0 * fetch_scale + write_kib * 1024.0 * write_scale,
        "trace_launch_ms_avg": sum(durs) / len(durs) / 1e6 if durs else None,
        "counter_launch_ms_avg": sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in fr)
        / len(fr) / 1e6,
        "vgpr": int(fr[0]["VGPR_Count"]),
        "scratch": int(fr[0]["Scratch_Size"]),
        "grid": int(fr[0]["Grid_Size"]),
        "kernel_stats": [{k: st[k] for k in ("Name", "Calls", "AverageNs", "Percentage")} for st in stats[:8]],
    }


def to_markdown(d, commands, bench_line=None):
    """Short text summary of `summarize`'s result, with the commands that made it."""
    L = [f"# {d['kernel']} — rocprofv3 summary", ""]
    L.append(f"Kernel sources hash `{d['source_hash']}`; launch configuration {json.dumps(d['launch'])}.")
    L.append("")
    L.append("## Commands")
    L.append("")
    L.append("```")
    L.extend(commands)
    L.append("```")
    L.append("")
    L.append("## Kernel trace (`--kernel-trace --stats`)")
    L.append("")
    L.append("| kernel | calls | average ns | % |")
    L.append("|---|---|---|---|")
    for st in d["kernel_stats"]:
        name = st["Name"].replace("(anonymous namespace)::", "").split("(vmc::")[0]
        L.append(f"| `{name}` | {st['Calls']} | {float(st['AverageNs']):.0f} | {float(st['Percentage']):.2f} |")
    L.append("")
    L.append(f"Average {d['kernel']} launch: {d['trace_launch_ms_avg']:.1f} ms over {d['dispatches']['trace']} "
             f"launches of the same size.")
    L.append("")
    L.append("## HBM traffic (`--pmc FETCH_SIZE`, then `--pmc WRITE_SIZE`)")
    L.append("")
    L.append("| quantity | value |")
    L.append("|---|---|")
    L.append(f"| FETCH_SIZE per launch (KiB) | {d['fetch_kib_per_launch']:.6g} |")
    L.append(f"| WRITE_SIZE per launch (KiB) | {d['write_kib_per_launch']:.6g} |")
    L.append(f"| copy calibration: bytes per FETCH_SIZE KiB / 1024 | {d['fetch_scale']:.4f} |")
    L.append(f"| copy calibration: bytes per WRITE_SIZE KiB / 1024 | {d['write_scale']:.4f} |")
    L.append(f"| HBM bytes per launch (scaled) | {d['hbm_bytes_per_launch']:.4g} |")
    L.append(f"| launch duration under counters (ms) | {d['counter_launch_ms_avg']:.1f} |")
    L.append(f"| VGPRs / scratch bytes per lane / grid | {d['vgpr']} / {d['scratch']} / {d['grid']} |")
    if bench_line:
        b = json.loads(bench_line)
        rf = b.get("roofline", {})
        L.append("")
        L.append("## bench.py line of the same configuration")
        L.append("")
        L.append(f"value {b['value']:.0f} {b['unit']}; roofline achieved {rf.get('achieved', 0):.0f} GB/s "
                 f"(frac {rf.get('frac', 0):.3f}); algorithmic bytes per launch "
                 f"{rf.get('alg_bytes_per_launch', 0):.4g}; event-timed launch {rf.get('launch_ms_avg', 0):.1f} ms.")
        if rf.get("alg_bytes_per_launch"):
            L.append(f"Measured / algorithmic bytes = {d['hbm_bytes_per_launch'] / rf['alg_bytes_per_launch']:.3f}.")
    return "\n".join(L) + "\n"


PHASE_ORDER = ("spmv", "lsolve", "usolve", "updates", "resid64")


def summarize_phases(trace, fetch, write, copy_fetch, copy_write, bench_log, hbm_peak_gbs=8000.0):
    """Per-phase figures of ``bench.py --phases`` runs: the k_phase launches in
    the order bench.py issues them (per path, the phases of PHASE_ORDER that it
    runs), each with its traced duration, its algorithmic bytes (from the bench
    line: rate times event-timed duration) and its HBM bytes (FETCH_SIZE and
    WRITE_SIZE scaled by the 1 GiB copy)."""
    cf = _largest_dispatch(_rows(copy_fetch, "counter_collection.csv"), "copyBuffer")[1]
    cw = _largest_dispatch(_rows(copy_write, "counter_collection.csv"), "copyBuffer")[1]
    fetch_scale = COPY_BYTES / (float(cf["Counter_Value"]) * 1024.0)
    write_scale = COPY_BYTES / (float(cw["Counter_Value"]) * 1024.0)
    line = None
    for ln in open(bench_log):
        if ln.startswith("{"):
            line = json.loads(ln)
    labels = []
    for path, res in line["phases"].items():
        labels += [(path, ph, res[ph]) for ph in PHASE_ORDER if ph in res]
    tr = _dispatches(_rows(trace, "kernel_trace.csv"), "k_phase")
    fr = _dispatches(_rows(fetch, "counter_collection.csv"), "k_phase")
    wr = _dispatches(_rows(write, "counter_collection.csv"), "k_phase")
    if not (len(tr) == len(fr) == len(wr) == len(labels)):
        raise ValueError(f"{len(labels)} phases in the bench line, dispatches: trace {len(tr)}, "
                         f"fetch {len(fr)}, write {len(wr)}")
    out = {"fetch_scale": fetch_scale, "write_scale": write_scale, "workload": line.get("workload"),
           "walkers": line.get("walkers"), "phases": []}
    for (path, ph, b), t, f, w in zip(labels, tr, fr, wr):
        ns = int(t["End_Timestamp"]) - int(t["Start_Timestamp"])
        alg = b["alg_gbs"] * b["ms"] * 1e6
        hbm = (float(f["Counter_Value"]) * fetch_scale + float(w["Counter_Value"]) * write_scale) * 1024.0
        out["phases"].append({
            "path": path, "phase": ph, "trace_ms": ns / 1e6, "event_ms": b["ms"], "us_per_rep": b["us_per_rep"],
            "alg_bytes": alg, "hbm_bytes": hbm, "alg_gbs": alg / ns, "hbm_gbs": hbm / ns,
            "alg_frac": alg / ns / hbm_peak_gbs, "hbm_frac": hbm / ns / hbm_peak_gbs})
    return out


def phases_markdown(d, commands):
    L = [f"# k_phase — per-phase HBM rates, {d['workload']} ({d['walkers']} walkers)", ""]
    L.append("Every walker's workgroup repeats one phase of the solve at the walker's real shape "
             "(one launch per phase and path). Algorithmic bytes are the method's own (the "
             "bench line's rate times its event-timed duration); HBM bytes are FETCH_SIZE and "
             f"WRITE_SIZE scaled by a 1 GiB device copy (x{d['fetch_scale']:.4f} and "
             f"x{d['write_scale']:.4f}). Both rates use the traced launch duration; peak 8 TB/s.")
    L += ["", "## Commands", "", "```"] + commands + ["```", ""]
    L += ["| path | phase | traced ms | µs per repeat | algorithmic GB/s (of peak) | HBM GB/s (of peak) | "
          "HBM / algorithmic |", "|---|---|---|---|---|---|---|"]
    for p in d["phases"]:
        L.append(f"| {p['path']} | {p['phase']} | {p['trace_ms']:.3f} | {p['us_per_rep']:.1f} | "
                 f"{p['alg_gbs']:.0f} ({p['alg_frac'] * 100:.0f}%) | {p['hbm_gbs']:.0f} ({p['hbm_frac'] * 100:.0f}%) | "
                 f"{p['hbm_bytes'] / p['alg_bytes']:.2f} |")
    return "\n".join(L) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sp = ap.add_subparsers(dest="cmd")
    q = sp.add_parser("phases")
    for k in ("trace", "fetch", "write", "copy_fetch", "copy_write", "bench_log", "out_md"):
        q.add_argument("--" + k.replace("_", "-"), required=True)
    q.add_argument("--commands", default=None, help="text file holding the profiling commands")
    s = sp.add_parser("summarize")
    for k in ("trace", "fetch", "write", "copy_fetch", "copy_write"):
        s.add_argument("--" + k.replace("_", "-"), required=True)
    s.add_argument("--prec", type=int, default=1)
    s.add_argument("--block", type=int, required=True, help="steps per launch in the profiled run")
    s.add_argument("--walkers", type=int, required=True)
    s.add_argument("--m-max", type=int, required=True)
    s.add_argument("--autotune", type=int, required=True, help="1 if the run autotuned (bench.py --autotune)")
    s.add_argument("--out-json", required=True)
    s.add_argument("--out-md", default=None)
    s.add_argument("--commands", default=None, help="text file holding the profiling commands")
    s.add_argument("--bench-log", default=None, help="bench.py output of the same configuration")
    args = ap.parse_args()
    if args.cmd == "phases":
        d = summarize_phases(args.trace, args.fetch, args.write, args.copy_fetch, args.copy_write, args.bench_log)
        cmds = open(args.commands).read().splitlines() if args.commands else []
        with open(args.out_md, "w") as f:
            f.write(phases_markdown(d, cmds))
        print(json.dumps(d, indent=1))
        return
    if args.cmd != "summarize":
        ap.error("the commands are summarize and phases")
    launch = {"block": args.block, "walkers": args.walkers, "m_max": args.m_max, "autotune": args.autotune}
    out = summarize(args.trace, args.fetch, args.write, args.copy_fetch, args.copy_write, args.prec, launch)
    with open(args.out_json, "w") as f:
        json.dump(out, f, indent=1)
    if args.out_md:
        cmds = open(args.commands).read().splitlines() if args.commands else []
        line = None
        if args.bench_log:
            for ln in open(args.bench_log):
                if ln.startswith("{"):
                    line = ln
        with open(args.out_md, "w") as f:
            f.write(to_markdown(out, cmds, line))
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
