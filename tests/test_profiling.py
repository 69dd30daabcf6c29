"""The rocprofv3 summaries behind bench.py's `traffic` and profiles/ (CPU only):
synthetic CSV files in the layout rocprofv3 writes, with known counter values,
give the bytes and rates worked out by hand here."""
import csv
import json
import os

import pytest

from paper_1008_5113_amd import profiling

TRACE_FIELDS = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
PMC_FIELDS = ["Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp",
              "VGPR_Count", "Scratch_Size", "Grid_Size"]


def _write(d, name, fields, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, name), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow({k: r.get(k, 0) for k in fields})


def _pmc(name, value, t0, t1):
    return {"Kernel_Name": name, "Counter_Name": "X", "Counter_Value": value, "Start_Timestamp": t0,
            "End_Timestamp": t1, "VGPR_Count": 64, "Scratch_Size": 52, "Grid_Size": 262144}


def _copy_dirs(tmp, fetch_kib, write_kib):
    """Copy calibration: the 1 GiB copy read fetch_kib and wrote write_kib."""
    _write(tmp / "cf", "run_counter_collection.csv", PMC_FIELDS,
           [_pmc("fill", 5.0, 0, 1), _pmc("__amd_rocclr_copyBuffer", fetch_kib, 0, 10)])
    _write(tmp / "cw", "run_counter_collection.csv", PMC_FIELDS,
           [_pmc("__amd_rocclr_copyBuffer", write_kib, 0, 10)])


def test_step_kernel_summary(tmp_path):
    # a copy of 2^30 bytes reads 2^19 KiB by FETCH_SIZE (half the bytes) and
    # writes 2^20 KiB: scales 2.0 and 1.0
    _copy_dirs(tmp_path, float(1 << 19), float(1 << 20))
    k1, k0 = "void k_run<1>(args)", "void k_run<0>(args)"
    _write(tmp_path / "tr", "run_kernel_trace.csv", TRACE_FIELDS,
           [{"Kernel_Name": k1, "Start_Timestamp": 0, "End_Timestamp": 2_000_000},
            {"Kernel_Name": k0, "Start_Timestamp": 0, "End_Timestamp": 9_000_000},
            {"Kernel_Name": k1, "Start_Timestamp": 0, "End_Timestamp": 4_000_000}])
    _write(tmp_path / "tr", "run_kernel_stats.csv", ["Name", "Calls", "AverageNs", "Percentage"],
           [{"Name": k1, "Calls": 2, "AverageNs": 3e6, "Percentage": 40.0}])
    _write(tmp_path / "fe", "run_counter_collection.csv", PMC_FIELDS,
           [_pmc(k1, 100.0, 0, 3_000_000), _pmc(k0, 1e9, 0, 1), _pmc(k1, 300.0, 0, 3_000_000)])
    _write(tmp_path / "wr", "run_counter_collection.csv", PMC_FIELDS,
           [_pmc(k1, 10.0, 0, 1), _pmc(k1, 30.0, 0, 1)])
    d = profiling.summarize(str(tmp_path / "tr"), str(tmp_path / "fe"), str(tmp_path / "wr"),
                            str(tmp_path / "cf"), str(tmp_path / "cw"), 1, {"chunk": 8})
    assert d["fetch_scale"] == pytest.approx(2.0) and d["write_scale"] == pytest.approx(1.0)
    assert d["fetch_kib_per_launch"] == pytest.approx(200.0)      # mean of the k_run<1> dispatches
    assert d["write_kib_per_launch"] == pytest.approx(20.0)
    assert d["hbm_bytes_per_launch"] == pytest.approx(200 * 1024 * 2.0 + 20 * 1024 * 1.0)
    assert d["trace_launch_ms_avg"] == pytest.approx(3.0)         # (2 + 4) / 2 ms, k_run<0> left out
    assert d["dispatches"] == {"trace": 2, "fetch": 2, "write": 2}
    assert d["source_hash"] == profiling.kernel_source_hash()
    md = profiling.to_markdown(d, ["cmd a", "cmd b"])
    assert "cmd a" in md and "k_run<1>" in md


def test_phase_summary(tmp_path):
    _copy_dirs(tmp_path, float(1 << 19), float(1 << 20))
    names = ["void k_phase<1>(a)"] * 2 + ["void k_phase<0>(a)"]
    # bench line: mixed spmv and lsolve, fp64 spmv; alg bytes = alg_gbs * ms * 1e6
    line = {"phases": {"mixed": {"m_avg": 1.0, "spmv": {"ms": 2.0, "us_per_rep": 100.0, "alg_gbs": 1000.0},
                                 "lsolve": {"ms": 1.0, "us_per_rep": 50.0, "alg_gbs": 500.0}},
                       "fp64": {"spmv": {"ms": 4.0, "us_per_rep": 200.0, "alg_gbs": 1000.0}}},
            "workload": "w", "walkers": 2}
    log = tmp_path / "ph.log"
    log.write_text("[bench] noise\n" + json.dumps(line) + "\n")
    durs = [2_000_000, 1_000_000, 4_000_000]
    _write(tmp_path / "tr", "run_kernel_trace.csv", TRACE_FIELDS,
           [{"Kernel_Name": "void k_run<1>(a)", "Start_Timestamp": 0, "End_Timestamp": 5}] +
           [{"Kernel_Name": k, "Start_Timestamp": 0, "End_Timestamp": t} for k, t in zip(names, durs)])
    fetch = [1e6, 2.5e5, 2e6]
    _write(tmp_path / "fe", "run_counter_collection.csv", PMC_FIELDS,
           [_pmc(k, v, 0, 1) for k, v in zip(names, fetch)])
    _write(tmp_path / "wr", "run_counter_collection.csv", PMC_FIELDS,
           [_pmc(k, 0.0, 0, 1) for k in names])
    d = profiling.summarize_phases(str(tmp_path / "tr"), str(tmp_path / "fe"), str(tmp_path / "wr"),
                                   str(tmp_path / "cf"), str(tmp_path / "cw"), str(log))
    got = [(p["path"], p["phase"]) for p in d["phases"]]
    assert got == [("mixed", "spmv"), ("mixed", "lsolve"), ("fp64", "spmv")]
    p0 = d["phases"][0]
    assert p0["alg_bytes"] == pytest.approx(1000.0 * 2.0 * 1e6)
    assert p0["alg_gbs"] == pytest.approx(1000.0)                 # same duration in trace and bench
    assert p0["hbm_bytes"] == pytest.approx(1e6 * 1024 * 2.0)
    assert p0["hbm_gbs"] == pytest.approx(1e6 * 1024 * 2.0 / 2e6)
    assert p0["hbm_frac"] == pytest.approx(p0["hbm_gbs"] / 8000.0)
    md = profiling.phases_markdown(d, ["c"])
    assert md.count("\n| mixed |") == 2 and "| fp64 | spmv |" in md
    # a dispatch count that does not match the bench line is an error
    _write(tmp_path / "fe", "run_counter_collection.csv", PMC_FIELDS, [_pmc(names[0], 1.0, 0, 1)])
    with pytest.raises(ValueError):
        profiling.summarize_phases(str(tmp_path / "tr"), str(tmp_path / "fe"), str(tmp_path / "wr"),
                                   str(tmp_path / "cf"), str(tmp_path / "cw"), str(log))
