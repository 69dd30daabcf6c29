"""Chained geometric reorders (Section 3.1: each reorder renumbers the order
the previous one left) and the two stop rules of the ratio solves, through the
C-ABI, on small systems."""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle.chain import StepRecord, replay
from oracle.reorder import geometric_reorder

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def vm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1008_5113_amd as vm
    vm.lib()  # fails loudly when the library is missing
    return vm


def _records(log_row):
    return [StepRecord(int(r["step"]), int(r["particle"]), np.array(r["new_pos"]), float(r["ratio"]),
                       float(r["u_acc"]), bool(r["flags"] & 1)) for r in log_row]


def test_reorder_chained_bitexact(vm):
    """A second reorder at the same positions, and one after a stretch of
    steps, start from the order the previous one left; the oracle is given
    that order and must agree exactly."""
    _say("case: chained reorders, sc 4x4x8, 2 walkers")
    inst = wl.small_instance(lattice=(4, 4, 8), cutoff=2.0, n_walkers=2, jitter=0.45)
    s = inst.systems[0]
    ctx = vm.Context.from_instance(inst)
    ctx.ilutp(reorder=True)
    first = [ctx.state(w) for w in range(2)]
    for w in range(2):
        row, col = geometric_reorder(inst.walkers[w].pos0, s)
        assert np.array_equal(first[w]["reorder_row"], row) and np.array_equal(first[w]["reorder_col"], col)
    ctx.ilutp(reorder=True)
    for w in range(2):
        st = ctx.state(w)
        row, col = geometric_reorder(inst.walkers[w].pos0, s, first[w]["reorder_row"], first[w]["reorder_col"])
        assert np.array_equal(st["reorder_row"], row) and np.array_equal(st["reorder_col"], col)
    ctx.run_steps(3 * s.n)
    ctx.sync()
    before = [ctx.state(w) for w in range(2)]
    ctx.ilutp(reorder=True)
    for w in range(2):
        st = ctx.state(w)
        row, col = geometric_reorder(before[w]["pos"], s, before[w]["reorder_row"], before[w]["reorder_col"])
        assert np.array_equal(st["reorder_row"], row) and np.array_equal(st["reorder_col"], col)
        # rows in reorder order; columns further permuted by the factorisation's pivots
        assert np.array_equal(st["row_particle"], row)
        assert np.array_equal(np.sort(st["col_site"]), np.arange(s.n))
    ctx.close()


@pytest.mark.parametrize("which", ["p_like_n4000", "jittered_n8192"])
def test_reorder_cell_search_bitexact(vm, which):
    """At n = 4000 and 8192 the first steps of a reorder search lattice cells
    around the particle and the orbital instead of scanning every free
    position; the permutation must still be the oracle's exactly, from the
    identity and chained after a stretch of steps (jittered sites and
    lognormal widths in the second case)."""
    _say(f"case: cell-search reorder {which}")
    if which == "p_like_n4000":
        inst = wl.mixed_n4000(n_walkers=1)
    else:
        inst = wl.stress_n8192(n_walkers=1)
    s = inst.systems[0]
    ctx = vm.Context.from_instance(inst)
    ctx.ilutp(reorder=True)
    st = ctx.state(0)
    row, col = geometric_reorder(inst.walkers[0].pos0, s)
    assert np.array_equal(st["reorder_row"], row) and np.array_equal(st["reorder_col"], col)
    ctx.run_steps(400)
    ctx.sync()
    before = ctx.state(0)
    ctx.ilutp(reorder=True)
    st = ctx.state(0)
    row, col = geometric_reorder(before["pos"], s, before["reorder_row"], before["reorder_col"])
    assert np.array_equal(st["reorder_row"], row) and np.array_equal(st["reorder_col"], col)
    ctx.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_plain_stop_against_ratio_relative_stop(vm, precision):
    """The same chain with the default stop (iterate on to tol * min(1,
    |ratio|)) and with plain_stop (stop at tol): every solve converged, no
    more iterations with plain_stop, and both replayed by the dense-LU oracle
    (the plain stop to a bound scaled by 1 / min(1, |ratio|))."""
    _say(f"case: stop rules, plain_n128, precision={precision}")
    inst = wl.plain_n128()
    s = inst.systems[0]
    w = inst.walkers[0]
    logs = {}
    for plain in (0, 1):
        ctx = vm.Context.from_instance(inst, precision=precision, plain_stop=plain)
        ctx.ilutp(reorder=True)
        logs[plain] = ctx.run_steps_logged(s.n)[0]
        st = ctx.stats()[0]
        ctx.close()
        assert st["status"] == 0
        assert np.all(logs[plain]["flags"] & vm.FLAG_CONVERGED)
    tol = inst.params.refine_tol if precision == vm.PREC_MIXED else inst.params.gmres_rtol
    for plain in (0, 1):
        rep = replay(s, w.pos0, w.seed, inst.params.step, _records(logs[plain]))
        r = np.abs(np.asarray(rep.oracle_ratios))
        d = np.abs(np.log(np.abs(logs[plain]["ratio"])) - np.log(r))
        # |d ln ratio| <~ ||r|| ||A^-T u|| / |ratio|: with the ratio-relative stop
        # the bound is tol-sized; with the plain stop it grows as 1 / |ratio|
        bound = 1e-10 if not plain else 1e-10 / np.minimum(1.0, r)
        _say(f"  plain_stop={plain}: iterations {logs[plain]['iters'].sum()}, max |d ln ratio| {d.max():.2e}, "
             f"min |ratio| {r.min():.2e}; {rep.summary()}")
        assert rep.pos_mismatch == 0 and rep.decision_mismatch_outside_tol == 0
        assert np.all(d <= 10 * bound)
    # the chains agree while they coincide; plain never iterates more on the same step
    k = 0
    a, b = logs[0], logs[1]
    while k < s.n and np.array_equal(a["new_pos"][k], b["new_pos"][k]) and (a["flags"][k] & 1) == (b["flags"][k] & 1):
        k += 1
    assert k > s.n // 2
    first = min(k, np.argmax(a["flags"][:k] & vm.FLAG_REORDERED) if np.any(a["flags"][:k] & vm.FLAG_REORDERED) else k)
    assert np.all(b["iters"][:first] <= a["iters"][:first])
    _ = tol
