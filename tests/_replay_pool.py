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


def replay_walkers(workload, step, starts, logs, procs, mode="sm", parts=1):
    """Replay walker w's log from positions starts[w] (dict walker -> array) in
    `procs` processes; returns {walker: ReplayReport}.  With parts > 1 each log
    is cut into that many consecutive pieces, each replayed from the positions
    the log itself gives at its start (a fresh inverse per piece), and the
    pieces' reports are merged in order."""
    from oracle.chain import ReplayReport, StepRecord, positions_after
    jobs = []
    for w, log in logs.items():
        recs = [(int(r["step"]), int(r["particle"]), tuple(r["new_pos"]), float(r["ratio"]),
                 float(r["u_acc"]), bool(r["flags"] & 1)) for r in log]
        cut = [len(recs) * k // parts for k in range(parts + 1)]
        pos = np.array(starts[w], dtype=np.float64)
        for k in range(parts):
            piece = recs[cut[k]:cut[k + 1]]
            jobs.append((workload, w, pos.copy(), step, piece, mode))
            pos = positions_after(pos, [StepRecord(*r) for r in piece])
    ctx = mp.get_context("spawn")
    with ctx.Pool(min(procs, len(jobs))) as pool:
        done = pool.map(_replay_one, jobs)
    out = {}
    for w, rep in done:  # pool.map keeps the job order: pieces in order
        m = out.setdefault(w, ReplayReport())
        m.steps += rep.steps
        m.max_dlog = max(m.max_dlog, rep.max_dlog)
        m.dlogs += rep.dlogs
        m.pos_mismatch += rep.pos_mismatch
        m.sign_mismatch += rep.sign_mismatch
        m.decision_mismatch += rep.decision_mismatch
        m.decision_mismatch_outside_tol += rep.decision_mismatch_outside_tol
        m.oracle_ratios += rep.oracle_ratios
    return out
