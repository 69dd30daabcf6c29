"""Benchmark: determinant-ratio steps/s of the persistent fused HIP path.

One bench step is one launch of the persistent step kernel in which every
walker of the batch takes ``--block`` Metropolis steps (proposal, Slater row,
ILUTP-preconditioned GMRES ratio, decision, row replacement, preconditioner
update, and any triggered reorder/refactor).  The launch is captured once in a
HIP graph and replayed.  Set-up (context creation, initial reorder and ILUTP),
the autotuner's trial (one launch of the same size) and W warm-up bench steps
are untimed; the K timed bench steps are bracketed by device synchronisations
and timed with events on the stream the kernel runs on, one event pair per
launch.  Every launch of the step kernel in a run has the same size, so a
profiler's per-launch average is the timed launches' duration.

After the timed region one more launch of the same size logs walkers 0 and 1
of each path; the two paths' ratios on those steps are compared with each
other, and the oracle leg recomputes sampled ones by dense LU.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "det-ratio steps/s, n=4000 x 512 walkers, mixed vs FP64 GMRES; % HBM peak"
HBM_PEAK_GBS = 8000.0


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# Algorithmic bytes of the method per timed region: every GMRES iteration
# streams A, L and U once (values + 2-byte column positions), the stored
# update vectors once, and a handful of n-vectors; a mixed-precision
# refinement pass streams A in FP64 once.
# ---------------------------------------------------------------------------
IDX = 2  # bytes per stored column position
def algorithmic_bytes(stats0, stats1, nnz, n, mixed: bool):
    """nnz = (nnz(A), nnz(L), nnz(U)) and n of every walker, or one triple and
    one n for all of them."""
    sv = 4 if mixed else 8
    k = len(stats0)
    ns = [n] * k if np.isscalar(n) else list(n)
    nnzs = [nnz] * k if np.isscalar(nnz[0]) else list(nnz)
    tot = 0.0
    for a, b, n, (nA, nL, nU) in zip(stats0, stats1, ns, nnzs):
        iters = b["iters"] - a["iters"]
        inner = b["inner_solves"] - a["inner_solves"]
        solves = b["solves"] - a["solves"]
        passes = b["refine_passes"] - a["refine_passes"]
        msum = b["update_sum"] - a["update_sum"]
        m_avg = msum / inner if inner else 0.0
        per_iter = (nA + nL + nU) * (sv + IDX) + n * sv * (1 + m_avg) + 4 * n * sv
        tot += iters * per_iter
        tot += inner * (n * 8)                   # solution accumulation write
        if mixed:
            tot += (solves + passes) * (nA * (8 + IDX) + n * 16)
    return tot


def measured_traffic(path, workload, launch):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE scaled by a plain-copy
    calibration), or None when that summary was taken on other kernel sources
    or another launch configuration."""
    from paper_1008_5113_amd.profiling import kernel_source_hash
    f = os.path.join(ROOT, "profiles", f"k_run_{workload}_{path}_counters.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        d = json.load(fh)
    same = d.get("source_hash") == kernel_source_hash() and d.get("launch") == launch
    return d["hbm_bytes_per_launch"] if same else None


def walker_nnz(ctx, nw: int):
    """Per-walker (nnz(A), nnz(L), nnz(U)) and n: the mean over up to two
    walkers of each size (walkers of one size have the same statistics)."""
    ns = [int(ctx.ns[w]) for w in range(nw)]
    by_n = {}
    for w, n in enumerate(ns):
        by_n.setdefault(n, []).append(w)
    per = {n: factor_nnz(ctx, ws[:2]) for n, ws in by_n.items()}
    return [per[n] for n in ns], ns


def factor_nnz(ctx, walkers):
    acc = np.zeros(3)
    for w in walkers:
        st = ctx.state(w, factors=True)
        acc += [st["a_len"].sum(), st["l_len"].sum(), st["u_len"].sum() + len(st["u_len"])]
    return acc / len(walkers)


def launch_plan(steps: int, warmup: int, block: int, autotune: bool):
    """The launches of one path, in order: (role, Metropolis steps per walker).
    Every launch has the same size, so the kernel's per-launch average under a
    profiler is the timed launches' duration."""
    if steps < 1 or warmup < 0 or block < 1:
        raise ValueError("steps >= 1, warmup >= 0 and block >= 1 are required")
    plan = []
    if autotune:
        plan.append(("autotune", block))
    plan += [("warmup", block)] * warmup
    plan += [("timed", block)] * steps
    plan.append(("logged", block))
    return plan


LOG_WALKERS = 2  # walkers whose records the post-timed launch keeps


def run_path(inst, precision, steps, warmup, block, walkers, stream_ptr, autotune=True, **kw):
    import torch
    import paper_1008_5113_amd as vm
    t0 = time.time()
    ctx = vm.Context.from_instance(inst, walkers=walkers, precision=precision, stream=stream_ptr, **kw)
    ctx.ilutp(reorder=True)
    ctx.sync()
    log(f"precision={precision}: set-up (create + reorder + ILUTP of {len(walkers)} walkers) "
        f"{time.time() - t0:.1f}s")
    plan = launch_plan(steps, warmup, block, autotune)
    tune = None
    if autotune:
        t1 = time.time()
        tune = ctx.autotune(trial_steps=block)
        log(f"precision={precision}: autotune (one trial launch of {block} steps) {time.time() - t1:.1f}s: {tune}")
    if warmup:
        t1 = time.time()
        for _ in range(warmup):
            ctx.run_steps(block, graph=True)
        ctx.sync()
        log(f"precision={precision}: warm-up {warmup} launches of {block} steps {time.time() - t1:.1f}s")
    s0 = ctx.stats()
    # one graph replay per bench step, each covering `block` steps of every
    # walker; one event pair per launch, recorded on the stream the kernel runs on
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    evs[0].record(stream)
    for k in range(steps):
        ctx.run_steps(block, graph=True)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    launch_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(steps)]
    ms = evs[0].elapsed_time(evs[steps])
    ctx.sync()
    s1 = ctx.stats()
    nnzw, nw_n = walker_nnz(ctx, len(walkers))
    nnz = factor_nnz(ctx, list(range(min(4, len(walkers)))))
    n = ctx.ns[0]
    # accuracy sample: one more launch of the same size logging walkers 0..1,
    # with their positions at its start (untimed)
    nlog = min(LOG_WALKERS, len(walkers))
    pos_before = [ctx.state(w)["pos"] for w in range(nlog)]
    logrec = ctx.run_steps_logged(block, log_walkers=nlog)
    bytes_ = algorithmic_bytes(s0, s1, nnzw, nw_n, precision == vm.PREC_MIXED)
    d = lambda k: sum(b[k] - a[k] for a, b in zip(s0, s1))  # noqa: E731
    nsteps = d("steps")
    ph = np.zeros(12)
    for a, b in zip(s0, s1):
        ph += np.array(b["phase_ticks"], dtype=np.float64) - np.array(a["phase_ticks"], dtype=np.float64)
    phase_us = {name: ph[k] / max(1, nsteps) / vm.vmcdet.WALL_CLOCK_HZ * 1e6
                for k, name in enumerate(vm.vmcdet.PHASE_NAMES)}
    # spread of the walkers' own time in the timed launches (the launch ends
    # with its slowest walker)
    kl = vm.vmcdet.PHASE_NAMES.index("launch")
    wt = np.array([b["phase_ticks"][kl] - a["phase_ticks"][kl] for a, b in zip(s0, s1)], dtype=np.float64)
    walker_tail = float(wt.max() / max(wt.mean(), 1.0))
    out = dict(
        ms=ms, launches=steps, launch_ms_avg=float(np.mean(launch_ms)),
        launch_ms_minmax=[float(np.min(launch_ms)), float(np.max(launch_ms))],
        steps=nsteps, steps_per_s=nsteps / (ms / 1e3),
        accept=d("accepted") / max(1, nsteps), iters_per_step=d("iters") / max(1, nsteps),
        inner_per_step=d("inner_solves") / max(1, nsteps), passes_per_step=d("refine_passes") / max(1, nsteps),
        reorders=d("reorders"), refactors=d("refactors"), ilu_retries=d("ilu_retries"),
        nonconverged=d("nonconverged"), walker_time_max_over_mean=walker_tail,
        max_N=max(b["max_N"] for b in s1), nnz_per_row=(nnz / n).tolist(),
        phase_us_per_walker_step={k: round(v, 2) for k, v in phase_us.items()},
        alg_bytes=bytes_, alg_bytes_per_launch=bytes_ / steps, autotune=tune,
        alg_gbs=bytes_ / (sum(launch_ms) / 1e3) / 1e9,
        launches_of_step_kernel=len(plan),
        status=[b["status"] for b in s1 if b["status"] != 0][:4])
    ctx.close()
    return out, {"pos0": pos_before, "log": logrec}


def path_agreement(la, lb):
    """Largest |ln|ratio_a| - ln|ratio_b|| over the steps the two paths' logs
    share with identical proposals (same step, particle and position), and the
    number of differing decisions among them."""
    best, diff, cnt = 0.0, 0, 0
    for ra, rb in zip(la.reshape(-1), lb.reshape(-1)):
        if ra["step"] != rb["step"] or ra["particle"] != rb["particle"] or \
                not np.array_equal(ra["new_pos"], rb["new_pos"]):
            break
        cnt += 1
        best = max(best, abs(np.log(abs(ra["ratio"])) - np.log(abs(rb["ratio"]))))
        diff += int((ra["flags"] & 1) != (rb["flags"] & 1))
    return {"steps_compared": cnt, "max_dlog": best, "decision_diff": diff}


# ---------------------------------------------------------------------------
# CPU baseline: the oracle's standard algorithm (explicit inverse with
# Sherman-Morrison updates), one walker per process, set-up untimed.
# ---------------------------------------------------------------------------
def _oracle_worker(args):
    workload, w, steps = args
    from threadpoolctl import threadpool_limits
    # import every BLAS user first: the limit applies to the libraries loaded
    # when it is set
    import scipy.linalg  # noqa: F401
    import workloads as wl
    from oracle.geometry import orbital_values, propose, slater_dense
    from oracle.ratio import StandardAlgorithm
    from oracle.rng import step_draws
    with threadpool_limits(1):
        inst = wl.WORKLOADS[workload](w + 1)
        s = inst.system_of(w)
        wk = inst.walkers[w]
        pos = wk.pos0.copy()
        sm = StandardAlgorithm(slater_dense(pos, s))
        t0 = time.perf_counter()
        for g in range(steps):
            p = g % s.n
            u = step_draws(wk.seed, g)
            rnew = propose(pos[p], u[:3], inst.params.step, s.box)
            row = orbital_values(rnew, s)
            ratio = sm.ratio(p, row)
            if ratio * ratio > u[3]:
                sm.accept(p, row, ratio)
                pos[p] = rnew
        return steps, time.perf_counter() - t0


def host_cpu():
    """CPU model and core counts of the host the oracle runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": avail}


CPU_PROC_CAP = 16  # worker processes at most (one GPU's share of the host)


def cpu_baseline(workload, procs, steps):
    import multiprocessing as mp
    host = host_cpu()
    if procs <= 0:
        procs = max(1, min(CPU_PROC_CAP, host["affinity"]))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        res = pool.map(_oracle_worker, [(workload, w, steps) for w in range(procs)])
    wall = time.perf_counter() - t0
    tot = sum(r[0] for r in res)
    loop = max(r[1] for r in res)
    return dict(value=tot / loop, unit="det-ratio steps/s", cores=procs, kind="oracle",
                sample=f"{workload}: walkers 0..{procs - 1}, {steps} steps each, one process per walker "
                       f"(single-threaded BLAS), standard algorithm (explicit inverse + Sherman-Morrison); "
                       f"inverse set-up untimed; wall {wall:.1f}s",
                host=host)


def oracle_accuracy(inst, logged, samples):
    """|ln|ratio_gpu| - ln|ratio_oracle|| on `samples` evenly spaced steps of
    each logged walker of each path, the oracle ratio by dense LU of the
    Slater matrix at the positions the log implies (its start positions and
    its accepted moves).  Part of the oracle leg."""
    from oracle.geometry import orbital_values, slater_dense
    from oracle.ratio import ratio_lu
    out = {}
    cache = {}
    for path, res in logged.items():
        worst, nchk = 0.0, 0
        for w, pos0 in enumerate(res["pos0"]):
            s = inst.system_of(w)
            recs = res["log"][w]
            pos = np.array(pos0, dtype=np.float64, copy=True)
            pick = set(np.linspace(0, len(recs) - 1, samples).round().astype(int).tolist())
            for k, r in enumerate(recs):
                p = int(r["particle"])
                rnew = np.array(r["new_pos"])
                if k in pick:
                    key = (w, int(r["step"]), pos.tobytes(), rnew.tobytes())
                    if key not in cache:
                        A = slater_dense(pos, s)
                        cache[key] = ratio_lu(A, p, orbital_values(rnew, s))[0]
                    ro = cache[key]
                    worst = max(worst, abs(np.log(abs(r["ratio"])) - np.log(abs(ro))))
                    nchk += 1
                if r["flags"] & 1:
                    pos[p] = rnew
        out[path] = {"steps_checked": nchk, "max_dlog": worst}
    return out


def copy_rate_gbs(nbytes=1 << 30, reps=5):
    """Bytes read plus written per second by a plain device-to-device copy of
    nbytes (the best of `reps` event-timed copies): what a streaming kernel
    reaches on this GPU, beside the published 8 TB/s."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        dst.copy_(src)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (best / 1e3) / 1e9


def phase_bench(inst, precision, walkers, stream_ptr, reps, warm_steps, **kw):
    """Per-phase micro-benchmarks at the workload's real shapes (one launch per
    phase, every walker's workgroup repeating the phase `reps` times)."""
    import torch
    import paper_1008_5113_amd as vm
    ctx = vm.Context.from_instance(inst, walkers=walkers, precision=precision, stream=stream_ptr, **kw)
    ctx.ilutp(reorder=True)
    if warm_steps:
        ctx.run_steps(warm_steps)
    ctx.sync()
    nnz = factor_nnz(ctx, list(range(min(4, len(walkers)))))
    n = ctx.ns[0]
    m_avg = float(np.mean([ctx.state(w)["n_updates"] for w in range(min(8, len(walkers)))]))
    nA, nL, nU = nnz
    sv = 4 if precision == vm.PREC_MIXED else 8
    per_rep = {
        "spmv": nA * (sv + IDX) + n * (4 + sv),
        "lsolve": (nL) * (sv + IDX) + n * 4,
        "usolve": (nU - n) * (sv + IDX) + n * (4 + sv),
        "updates": m_avg * n * sv,
        "resid64": nA * (8 + IDX) + n * (4 + 8 + 8),
    }
    out = {"m_avg": m_avg, "nnz_per_row": (nnz / n).tolist()}
    stream = torch.cuda.current_stream()
    for ph in ["spmv", "lsolve", "usolve", "updates", "resid64"]:
        if ph == "resid64" and precision != vm.PREC_MIXED:
            continue
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        ctx.phase_bench(ph, reps)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        b = per_rep[ph] * reps * len(walkers)
        out[ph] = {"ms": ms, "us_per_rep": ms * 1e3 / reps, "alg_gbs": b / (ms / 1e3) / 1e9,
                   "frac_hbm": b / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}
        log(f"phase {ph}: {out[ph]}")
    ctx.close()
    return out


def scaling_point(lattice, n_walkers, stream_ptr, args):
    """Steps/s of both paths on an sc lattice of the n = 4000 workload's
    orbitals (Gaussian 0.35 plus the p-like term, cutoff 2.5), beside the HBM
    bound of the standard algorithm of Section 1 (explicit inverse, updated by
    Sherman-Morrison on every accepted move).  An accepted move rewrites the
    whole n x n FP64 inverse (read and write, 16 n^2 bytes); a rejected one
    reads about (2W + 1) n entries; so at acceptance a the dense step moves
    at least a 16 n^2 bytes and its rate is at most 8 TB/s / that."""
    import workloads as wl
    import paper_1008_5113_amd as vm
    s = wl.make_system(lattice, sigma=0.35, kind=wl.ORB_GAUSS_PX, p_scale=0.1, p_sigma=0.5, cutoff=2.5)
    ws = [wl.Walker(0, wl.initial_positions(s.sites, s.box, w, 0.3), w) for w in range(n_walkers)]
    inst = wl.Instance(f"sc{lattice[0]}x{lattice[1]}x{lattice[2]}", [s], ws,
                       wl.Params(step=0.25, mixed=True, m_max=96))
    out = {"workload": inst.name, "n": s.n, "walkers": n_walkers}
    walkers = list(range(n_walkers))
    for path, prec in (("mixed", vm.PREC_MIXED), ("fp64", vm.PREC_FP64)):
        r, _ = run_path(inst, prec, args.steps, args.warmup, args.block, walkers, stream_ptr,
                        autotune=bool(args.autotune), **({"m_max": args.m_max} if args.m_max else {}))
        out[path] = {"steps_per_s": r["steps_per_s"], "accept": r["accept"], "iters_per_step": r["iters_per_step"],
                     "alg_gbs": r["alg_gbs"]}
    acc = out["fp64"]["accept"]
    out["dense_standard_bound_steps_per_s"] = 8e12 / (acc * 16.0 * s.n * s.n)
    if args.dense_steps:
        out["dense_standard"] = dense_standard(inst, walkers, stream_ptr, args.dense_steps)
    return out


def dense_standard(inst, walkers, stream_ptr, steps):
    """The standard algorithm on the GPU (explicit inverse, Sherman-Morrison on
    accept): inverse built by the solver (untimed), one warm-up launch of 8
    steps, then `steps` timed steps of every walker in one launch."""
    import torch
    import paper_1008_5113_amd as vm
    ctx = vm.Context.from_instance(inst, walkers=walkers, precision=vm.PREC_FP64, stream=stream_ptr)
    t0 = time.time()
    ctx.ilutp(reorder=True)
    ctx.sm_prepare(1e-12)
    log(f"dense standard algorithm: inverses of {len(walkers)} walkers (n={ctx.ns[0]}) {time.time() - t0:.1f}s")
    ctx.sm_run_steps(8)
    s0 = ctx.stats()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    ctx.sm_run_steps(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    s1 = ctx.stats()
    ms = e0.elapsed_time(e1)
    ctx.close()
    nsteps = sum(b["steps"] - a["steps"] for a, b in zip(s0, s1))
    nacc = sum(b["accepted"] - a["accepted"] for a, b in zip(s0, s1))
    n = inst.systems[0].n
    bytes_ = nacc * 16.0 * n * n
    return {"steps_per_s": nsteps / (ms / 1e3), "accept": nacc / max(1, nsteps),
            "inverse_update_gbs": bytes_ / (ms / 1e3) / 1e9}


def energy_bench(inst, walkers, stream_ptr, args):
    """Kinetic-energy terms (Section 2.3, eq. (energyEq)) through the solver:
    after the step warm-up (so the preconditioner carries stored updates),
    one timed vmc_kinetic_energy call over particles [0, P) of every walker.
    Each term is one more determinant-ratio solve."""
    import torch
    import paper_1008_5113_amd as vm
    prec = vm.PREC_MIXED if inst.params.mixed else vm.PREC_FP64
    kw = {"m_max": args.m_max} if args.m_max else {}
    if args.energy_tol > 0:
        kw["energy_tol"] = args.energy_tol
    ctx = vm.Context.from_instance(inst, stream=stream_ptr, precision=prec, **kw)
    ctx.ilutp(reorder=True)
    tune = ctx.autotune(trial_steps=args.block) if args.autotune else None
    if args.warmup:
        ctx.run_steps(args.warmup * args.block)
    ctx.sync()
    P = args.energy_particles
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0 = ctx.stats()
    torch.cuda.synchronize()
    e0.record(stream)
    energies = ctx.kinetic_energy(p_begin=0, p_end=P)
    e1.record(stream)
    torch.cuda.synchronize()
    s1 = ctx.stats()
    ms = e0.elapsed_time(e1)
    nnz = factor_nnz(ctx, list(range(min(4, len(walkers)))))
    n = ctx.ns[0]
    ctx.close()
    bytes_ = algorithmic_bytes(s0, s1, nnz, n, prec == vm.PREC_MIXED)
    d = lambda k: sum(b[k] - a[k] for a, b in zip(s0, s1))  # noqa: E731
    terms = len(walkers) * P
    gbs = bytes_ / (ms / 1e3) / 1e9
    return {
        "metric": "kinetic-energy terms per second (one GMRES solve each)",
        "value": terms / (ms / 1e3), "unit": "terms/s", "n_gpus": 1, "ms": ms,
        "higher_is_better": True, "dtype": "fp32+fp64" if prec == vm.PREC_MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": inst.name, "walkers": len(walkers), "n": n, "particles_per_walker": P,
                   "warmup_steps": args.warmup * args.block, "autotune": bool(args.autotune),
                   "energy_tol": args.energy_tol if args.energy_tol > 0 else "ratio solves'"},
        "iters_per_term": d("iters") / terms, "inner_per_term": d("inner_solves") / terms,
        "refine_per_term": d("refine_passes") / terms, "reorders": d("reorders"),
        "energy_partial_mean": float(np.mean(energies)),
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                     "frac": gbs / 8000.0, "traffic": None,
                     "kernel": f"k_energy<{1 if prec == vm.PREC_MIXED else 0}>, one launch"},
        "autotune_info": tune,
    }


BLOCK = 200       # Metropolis steps of every walker per bench step (one launch)
STEPS = 20        # timed bench steps
WARMUP = 5        # untimed bench steps before them
ORACLE_SAMPLES = 4  # logged steps per walker recomputed by the oracle


def parse_args(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=STEPS, help="timed bench steps (launches)")
    ap.add_argument("--warmup", type=int, default=WARMUP, help="untimed bench steps (launches) before them")
    ap.add_argument("--block", type=int, default=BLOCK,
                    help="Metropolis steps of every walker per bench step (one launch of the step kernel)")
    ap.add_argument("--workload", default="mixed_n4000")
    ap.add_argument("--walkers", type=int, default=0, help="0: the workload's count")
    ap.add_argument("--paths", default="mixed,fp64")
    ap.add_argument("--m-max", type=int, default=0,
                    help="cap on stored updates (0: the workload's, or 200 when autotuning)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: run the cost-balance autotuner before warm-up, over one trial launch of --block "
                         "steps (the same size as every other launch); 0: refactor after a fixed m_max "
                         "updates only")
    ap.add_argument("--cpu-procs", type=int, default=0, help="oracle processes (0: the host's cores, at most 16)")
    ap.add_argument("--cpu-steps", type=int, default=60)
    ap.add_argument("--oracle-samples", type=int, default=ORACLE_SAMPLES)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--phases", action="store_true", help="per-phase micro-benchmarks only")
    ap.add_argument("--phase-reps", type=int, default=20)
    ap.add_argument("--energy", action="store_true",
                    help="time the kinetic energy through the solver instead of the step")
    ap.add_argument("--energy-particles", type=int, default=128,
                    help="particles per walker in the timed kinetic-energy call")
    ap.add_argument("--energy-tol", type=float, default=0.0,
                    help="residual tolerance of the kinetic-energy solves (0: the ratio solves')")
    ap.add_argument("--scaling", default="",
                    help="comma-separated sc lattices like 6x6x12,8x8x16: FP64 and mixed steps/s per n "
                         "beside the HBM bound of the dense standard algorithm")
    ap.add_argument("--dense-steps", type=int, default=100,
                    help="with --scaling: timed steps of the GPU standard algorithm (0: skip)")
    ap.add_argument("--gather-calibration", action="store_true",
                    help="random 128-byte-row and 4-byte-word gathers of known size, for the HBM counters")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args(argv)
    if args.steps < 1 or args.warmup < 0 or args.block < 1:
        ap.error("--steps >= 1, --warmup >= 0 and --block >= 1 are required")
    if not args.m_max and args.autotune:
        args.m_max = 200  # a cap only: the tuned cost balance decides when to refactor
    return args


def main(argv=None):
    args = parse_args(argv)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: walkers are independent chains, so the benchmark "
              "measures one GPU's share of them; use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.gather_calibration:
        # gathers whose bytes are known: K random 128-byte lines read whole
        # (index_select of rows), then one 4-byte word from each of K random
        # lines (the fetch granularity decides what HBM moves for it)
        import torch
        lines, K = (1 << 30) // 128, 1 << 22
        src = torch.ones(lines, 32, dtype=torch.float32, device="cuda")
        g = torch.Generator(device="cuda")
        g.manual_seed(7)
        idx = torch.randperm(lines, device="cuda", generator=g)[:K].contiguous()
        flat = src.view(-1)
        torch.cuda.synchronize()
        for _ in range(3):
            rows = torch.index_select(src, 0, idx)
            words = flat[idx * 32]
        torch.cuda.synchronize()
        print(json.dumps({"lines": lines, "gathered_lines": K, "row_bytes": 128, "word_bytes": 4,
                          "index_bytes": 8, "launches": 3, "check": float(rows.sum() + words.sum())}))
        return
    if args.copy_calibration:
        import torch
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 3}))
        return
    import torch
    import workloads as wl
    import paper_1008_5113_amd as vm
    torch.cuda.set_device(0)
    inst = wl.WORKLOADS[args.workload]() if not args.walkers else wl.WORKLOADS[args.workload](args.walkers)
    nw = len(inst.walkers)
    walkers = list(range(nw))
    stream_ptr = torch.cuda.current_stream().cuda_stream
    if args.energy:
        print(json.dumps(energy_bench(inst, walkers, stream_ptr, args)))
        return
    if args.scaling:
        for lat in args.scaling.split(","):
            print(json.dumps(scaling_point(tuple(int(x) for x in lat.split("x")), nw, stream_ptr, args)),
                  flush=True)
        return
    if args.phases:
        res = {}
        for path in args.paths.split(","):
            prec = vm.PREC_MIXED if path == "mixed" else vm.PREC_FP64
            kw = {"m_max": args.m_max} if args.m_max else {}
            res[path] = phase_bench(inst, prec, walkers, stream_ptr, args.phase_reps, args.warmup * args.block, **kw)
        print(json.dumps({"phases": res, "workload": args.workload, "walkers": nw}))
        return
    results, logged = {}, {}
    for path in args.paths.split(","):
        prec = vm.PREC_MIXED if path == "mixed" else vm.PREC_FP64
        log(f"path {path}: {nw} walkers, n={inst.systems[0].n}, {args.steps} timed launches of {args.block} steps")
        kw = {"m_max": args.m_max} if args.m_max else {}
        results[path], logged[path] = run_path(inst, prec, args.steps, args.warmup, args.block, walkers,
                                               stream_ptr, autotune=bool(args.autotune), **kw)
        log(f"path {path}: {json.dumps(results[path])}")
    head = results.get("mixed") or results[next(iter(results))]
    headpath = "mixed" if "mixed" in results else next(iter(results))
    launch = {"block": args.block, "walkers": nw, "m_max": args.m_max or inst.params.m_max,
              "autotune": args.autotune}
    sizes = sorted({s.n for s in inst.systems})
    metric = METRIC if args.workload == "mixed_n4000" else \
        f"det-ratio steps/s, {args.workload} (n = {', '.join(map(str, sizes))}) x {nw} walkers; % HBM peak"
    out = {
        "metric": metric,
        "value": head["steps_per_s"],
        "unit": "det-ratio steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if headpath == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": sizes[0] if len(sizes) == 1 else sizes, "walkers": nw,
                   "step": f"one graph-replayed launch of the step kernel: {args.block} Metropolis steps of "
                           f"every walker ({args.block * nw} det-ratio steps)",
                   "refactor": (f"cost balance, autotuned over one trial launch of {args.block} steps, "
                                f"cap {args.m_max}" if args.autotune
                                else f"every {args.m_max or inst.params.m_max} updates"),
                   "lattice": ",".join(dict.fromkeys("x".join(str(x) for x in s.lattice) for s in inst.systems)),
                   "path": headpath},
        "paths": results,
    }
    if "mixed" in results and "fp64" in results:
        out["mixed_over_fp64"] = results["mixed"]["steps_per_s"] / results["fp64"]["steps_per_s"]
        out["mixed_vs_fp64"] = path_agreement(logged["mixed"]["log"], logged["fp64"]["log"])
    out["roofline"] = {"bound": "hbm", "achieved": head["alg_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": head["alg_gbs"] / HBM_PEAK_GBS,
                       "traffic": measured_traffic(headpath, args.workload, launch),
                       "kernel": f"k_run<{1 if headpath == 'mixed' else 0}> (persistent fused step kernel), "
                                 f"{args.block} steps x {nw} walkers per launch",
                       "launch_ms_avg": head["launch_ms_avg"],
                       "alg_bytes_per_launch": head["alg_bytes_per_launch"]}
    rf = out["roofline"]
    if rf["traffic"]:
        rf["traffic_gbs"] = rf["traffic"] / (head["launch_ms_avg"] / 1e3) / 1e9
    rf["copy_gbs"] = copy_rate_gbs()
    log(f"plain 1 GiB device copy: {rf['copy_gbs']:.0f} GB/s (bytes read + written)")
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle processes x {args.cpu_steps} steps; oracle check of "
            f"{args.oracle_samples} logged steps per walker")
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_procs, args.cpu_steps)
        acc = oracle_accuracy(inst, logged, args.oracle_samples)
        out["cpu_baseline"]["ratio_check"] = acc
        out["dlog_vs_oracle"] = {p: v["max_dlog"] for p, v in acc.items()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
