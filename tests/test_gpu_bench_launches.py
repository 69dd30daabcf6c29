"""Parity in the benchmark's own configuration and launch pattern: the n = 4000
workload with all 512 walkers, mixed precision, the autotuned cost balance
(one trial launch of 200 steps) and a cap of 200 stored updates, run as
bench.py runs it, in persistent launches of 200 steps.  Walkers 0..3 are
logged over twenty launches (4000 steps each, one full sweep) and replayed by
the oracle's standard algorithm (explicit inverse, Sherman-Morrison), in
pieces of 1000 steps, one host process per piece; the FP64 path runs the same
chains and its ratios are compared with the oracle's and the mixed path's
while the chains agree."""
import sys
import time

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

DLOG_TOL = 1e-10
DEC_TOL = 1e-9
LOGGED = 4
TRIAL = 200
CAP = 200
BLOCK = 200
LAUNCHES = 20
PARTS = 4  # replay pieces per walker, one host process each


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def vm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1008_5113_amd as vm
    vm.lib()
    return vm


def _run(vm, inst, precision):
    _say(f"  precision={precision}: create, ILUTP, autotune over {TRIAL} steps")
    ctx = vm.Context.from_instance(inst, precision=precision, m_max=CAP)
    try:
        ctx.ilutp(reorder=True)
        ctx.autotune(trial_steps=TRIAL)
        starts = {w: ctx.state(w)["pos"].copy() for w in range(LOGGED)}
        logs = {w: [] for w in range(LOGGED)}
        for k in range(LAUNCHES):
            _say(f"  precision={precision}: logged launch {k + 1} of {LAUNCHES} ({BLOCK} steps, {len(inst.walkers)} walkers)")
            log = ctx.run_steps_logged(BLOCK, log_walkers=LOGGED)
            for w in range(LOGGED):
                logs[w].append(log[w])
        st = ctx.stats()
    finally:
        ctx.close()
    assert all(s["status"] == 0 for s in st)
    return starts, {w: np.concatenate(v) for w, v in logs.items()}


def test_bench_launches_replayed(vm):
    from _replay_pool import replay_walkers
    inst = wl.mixed_n4000()
    _say(f"case: bench launch pattern, {len(inst.walkers)} walkers, walkers 0..{LOGGED - 1} over "
         f"{LAUNCHES} launches of {BLOCK} steps")
    starts, mixed = _run(vm, inst, vm.PREC_MIXED)
    starts64, fp64 = _run(vm, inst, vm.PREC_FP64)
    for w in range(LOGGED):
        assert len(mixed[w]) == LAUNCHES * BLOCK
        assert np.all(np.diff(mixed[w]["step"]) == 1)
        assert np.all(mixed[w]["flags"] & vm.FLAG_CONVERGED)
        assert np.all(fp64[w]["flags"] & vm.FLAG_CONVERGED)
    _say(f"  oracle replays of {LOGGED} walkers x {LAUNCHES * BLOCK} steps ({LOGGED * PARTS} processes)")
    t0 = time.time()
    reps = replay_walkers("mixed_n4000", inst.params.step, starts, mixed, LOGGED * PARTS, parts=PARTS)
    _say(f"  oracle replays {time.time() - t0:.1f}s")
    for w, rep in sorted(reps.items()):
        _say(f"  walker {w} mixed vs oracle: " + rep.summary())
        assert rep.pos_mismatch == 0
        assert rep.decision_mismatch_outside_tol == 0
        assert rep.max_dlog <= DLOG_TOL, (w, rep.max_dlog)
    for w in range(LOGGED):
        assert np.array_equal(starts[w], starts64[w])
        a, b = mixed[w], fp64[w]
        oracle = np.array(reps[w].oracle_ratios)
        k = 0
        while k < len(a) and a["step"][k] == b["step"][k] and np.array_equal(a["new_pos"][k], b["new_pos"][k]) \
                and (a["flags"][k] & 1) == (b["flags"][k] & 1):
            k += 1
        d_or = np.abs(np.log(np.abs(b["ratio"][:k])) - np.log(np.abs(oracle[:k])))
        d_mx = np.abs(np.log(np.abs(b["ratio"][:k])) - np.log(np.abs(a["ratio"][:k])))
        _say(f"  walker {w}: chains identical for {k} of {len(a)} steps; fp64 vs oracle max "
             f"{d_or.max() if k else 0:.2e}, fp64 vs mixed max {d_mx.max() if k else 0:.2e}")
        assert k > 0
        assert d_or.max() <= DLOG_TOL
        assert d_mx.max() <= DLOG_TOL
        if k < len(a):
            # the chains part only at a decision taken inside the tolerance
            assert abs(oracle[k] ** 2 - a["u_acc"][k]) <= DEC_TOL
