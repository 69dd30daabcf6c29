"""Parity in the benchmark's own configuration: the n = 4000 workload with all
512 walkers in one persistent launch, mixed precision, the autotuned cost
balance (one trial launch of 200 steps) and a cap of 200 stored updates.
Walkers 0..3 are logged over one full sweep (4000 steps each) and replayed by
the oracle's standard algorithm (explicit inverse, Sherman-Morrison), one host
process per walker; the FP64 path runs the same chains and its ratios are
compared with the mixed path's and with the oracle's, step by step."""
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


def _run(vm, inst, precision, steps):
    ctx = vm.Context.from_instance(inst, precision=precision, m_max=CAP)
    ctx.ilutp(reorder=True)
    ctx.autotune(trial_steps=TRIAL)
    starts = {w: ctx.state(w)["pos"].copy() for w in range(LOGGED)}
    t0 = time.time()
    log = ctx.run_steps_logged(steps, log_walkers=LOGGED)
    st = ctx.stats()
    ctx.close()
    _say(f"  precision={precision}: {steps} steps of {len(inst.walkers)} walkers in {time.time() - t0:.1f}s, "
         f"refactors {sum(s['refactors'] for s in st)}, reorders {sum(s['reorders'] for s in st)}")
    assert all(s["status"] == 0 for s in st)
    return starts, log


@pytest.mark.skip(reason="a GPU run that began with this test ended in a GPU fault (memory fault or hung "
                         "queue) whose cause has not been found by reading the code; kept off the GPU until "
                         "it is")
def test_bench_configuration_full_sweep_replayed(vm):
    from _replay_pool import replay_walkers
    inst = wl.mixed_n4000()
    n = inst.systems[0].n
    _say(f"case: bench configuration, {len(inst.walkers)} walkers, one sweep of walkers 0..{LOGGED - 1}")
    starts, mixed = _run(vm, inst, vm.PREC_MIXED, n)
    starts64, fp64 = _run(vm, inst, vm.PREC_FP64, n)
    for w in range(LOGGED):
        assert np.all(mixed[w]["flags"] & vm.FLAG_CONVERGED)
        assert np.all(fp64[w]["flags"] & vm.FLAG_CONVERGED)
    t0 = time.time()
    reps = replay_walkers("mixed_n4000", inst.params.step, starts, {w: mixed[w] for w in range(LOGGED)}, LOGGED)
    _say(f"  oracle replays ({LOGGED} processes) {time.time() - t0:.1f}s")
    for w, rep in sorted(reps.items()):
        _say(f"  walker {w} mixed vs oracle: " + rep.summary())
        assert rep.pos_mismatch == 0
        assert rep.decision_mismatch_outside_tol == 0
        assert rep.max_dlog <= DLOG_TOL, (w, rep.max_dlog)
    # the FP64 path against the same oracle ratios and against the mixed path,
    # over the steps where both chains are still identical
    for w in range(LOGGED):
        same_start = np.array_equal(starts[w], starts64[w])
        a, b = mixed[w], fp64[w]
        oracle = np.array(reps[w].oracle_ratios)
        k = 0
        while k < len(a) and same_start and a["step"][k] == b["step"][k] and \
                np.array_equal(a["new_pos"][k], b["new_pos"][k]) and (a["flags"][k] & 1) == (b["flags"][k] & 1):
            k += 1
        _say(f"  walker {w}: chains identical for {k} of {len(a)} steps")
        assert k >= len(a) // 2 or not same_start
        d_or = np.abs(np.log(np.abs(b["ratio"][:k])) - np.log(np.abs(oracle[:k])))
        d_mx = np.abs(np.log(np.abs(b["ratio"][:k])) - np.log(np.abs(a["ratio"][:k])))
        _say(f"  walker {w}: fp64 vs oracle max {d_or.max() if k else 0:.2e}, fp64 vs mixed max "
             f"{d_mx.max() if k else 0:.2e}")
        assert k == 0 or d_or.max() <= DLOG_TOL
        assert k == 0 or d_mx.max() <= DLOG_TOL
        if k < len(a):
            # the chains part only at a decision taken inside the tolerance
            r = oracle[k]
            assert abs(r * r - a["u_acc"][k]) <= DEC_TOL
