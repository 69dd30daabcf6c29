"""Parallel oracle replays for the GPU parity tests: one process per logged
walker, each with single-threaded BLAS (test infrastructure)."""
import multiprocessing as mp

import numpy as np


def _replay_one(args):
    workload, walker, pos0, step, recs, mode = args
    from threadpoolctl import threadpool_limits
    import scipy.linalg  # noqa: F401  (loaded before the thread limit applies)
    import workloads as wl
    from oracle.chain import StepRecord, replay
    with threadpool_limits(1):
        inst = wl.WORKLOADS[workload](walker + 1)
        s = inst.system_of(walker)
        log = [StepRecord(int(g), int(p), np.array(x), float(r), float(u), bool(a)) for g, p, x, r, u, a in recs]
        rep = replay(s, pos0, inst.walkers[walker].seed, step, log, mode=mode)
        return walker, rep


def replay_walkers(workload, step, starts, logs, procs, mode="sm"):
    """Replay walker w's log from positions starts[w] (dict walker -> array) in
    `procs` processes; returns {walker: ReplayReport}."""
    jobs = []
    for w, log in logs.items():
        recs = [(int(r["step"]), int(r["particle"]), tuple(r["new_pos"]), float(r["ratio"]),
                 float(r["u_acc"]), bool(r["flags"] & 1)) for r in log]
        jobs.append((workload, w, starts[w], step, recs, mode))
    ctx = mp.get_context("spawn")
    with ctx.Pool(min(procs, len(jobs))) as pool:
        return dict(pool.map(_replay_one, jobs))
