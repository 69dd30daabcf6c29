"""GPU parity for the standard algorithm (Section 1: explicit inverse,
Sherman-Morrison on accept), the comparison path, through the C-ABI.

The stored inverse is built column by column by the preconditioned solver to a
relative residual tol; a column then differs from the exact one by
A^{-1} r, so every entry is within ||A^{-1}||_2 ||r||_2 <= ||A^{-1}||_2 * 10 tol
(the factor 10 covers the FP64 path's recurrence estimate against the true
residual).  The steps are replayed by the oracle with dense LU: ratios to the
1e-10 bound in ln|ratio| of the sparse path, decisions equal outside 1e-9.
"""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle.chain import StepRecord, positions_after, replay
from oracle.geometry import slater_dense

pytestmark = pytest.mark.gpu

DLOG_TOL = 1e-10
DEC_TOL = 1e-9
TOL = 1e-13


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


@pytest.mark.parametrize("precision", [0, 1])
def test_inverse_matches_dense(vm, precision):
    _say(f"case: stored inverse plain_n128 precision={precision}")
    inst = wl.plain_n128()
    s = inst.systems[0]
    ctx = vm.Context.from_instance(inst, precision=precision)
    ctx.ilutp(reorder=True)
    ctx.sm_prepare(TOL)
    B = ctx.sm_inverse(0)
    ctx.close()
    A = slater_dense(inst.walkers[0].pos0, s)
    ref = np.linalg.inv(A)
    bound = 10.0 * TOL * np.linalg.norm(ref, 2)
    err = np.max(np.abs(B - ref))
    _say(f"  max |B - inv(A)| {err:.3e}, bound {bound:.3e}")
    assert err <= bound


def test_standard_steps_replay(vm):
    _say("case: standard-algorithm steps plain_n128, 2 sweeps")
    inst = wl.plain_n128()
    s = inst.systems[0]
    ctx = vm.Context.from_instance(inst)
    ctx.ilutp(reorder=True)
    ctx.sm_prepare(TOL)
    log = ctx.sm_run_steps(2 * s.n, log=True)
    pos_gpu = ctx.state(0)["pos"]
    stats = ctx.stats()[0]
    ctx.close()
    assert stats["status"] == 0 and stats["steps"] == 2 * s.n
    recs = _records(log[0])
    rep = replay(s, inst.walkers[0].pos0, inst.walkers[0].seed, inst.params.step, recs, dec_tol=DEC_TOL)
    _say(f"  {rep.summary()}; acceptance {np.mean([r.accepted for r in recs]):.3f}")
    assert rep.pos_mismatch == 0 and rep.sign_mismatch == 0
    assert rep.decision_mismatch_outside_tol == 0
    assert rep.max_dlog < DLOG_TOL
    assert np.array_equal(pos_gpu, positions_after(inst.walkers[0].pos0, recs))


def test_standard_full_size_sampled(vm):
    """n = 4000 (the benchmark's orbitals), 4 walkers, 60 steps; walker 0
    replayed by the oracle's own standard algorithm."""
    _say("case: standard algorithm n=4000, 4 walkers, 60 steps")
    inst = wl.mixed_n4000(4)
    s = inst.systems[0]
    ctx = vm.Context.from_instance(inst, precision=0)
    ctx.ilutp(reorder=True)
    ctx.sm_prepare(TOL)
    log = ctx.sm_run_steps(60, log=True)
    stats = ctx.stats()
    ctx.close()
    assert all(st["status"] == 0 for st in stats)
    rep = replay(s, inst.walkers[0].pos0, inst.walkers[0].seed, inst.params.step, _records(log[0]),
                 dec_tol=DEC_TOL, mode="sm")
    _say(f"  walker 0: {rep.summary()}")
    assert rep.pos_mismatch == 0 and rep.sign_mismatch == 0
    assert rep.decision_mismatch_outside_tol == 0
    assert rep.max_dlog < DLOG_TOL


def test_standard_requires_prepare(vm):
    inst = wl.plain_n128()
    ctx = vm.Context.from_instance(inst)
    with pytest.raises(vm.VmcError) as ei:
        ctx.sm_run_steps(1)
    assert ei.value.status == vm.VMC_ESTATE
    ctx.close()


def test_standard_and_sparse_state_guards(vm):
    """A stored inverse is refused once a sparse-path call has run after it; the
    sparse path is refused on walkers the standard algorithm moved until their
    rows and factors are rebuilt, and after the rebuild its ratios match the
    oracle from the moved positions."""
    _say("case: standard/sparse state guards plain_n128")
    inst = wl.plain_n128()
    s = inst.systems[0]
    ctx = vm.Context.from_instance(inst)
    ctx.ilutp(reorder=True)
    ctx.sm_prepare(TOL)
    ctx.run_steps(4)
    ctx.sync()
    with pytest.raises(vm.VmcError) as ei:
        ctx.sm_run_steps(1)
    assert ei.value.status == vm.VMC_ESTATE
    ctx.sm_prepare(TOL)
    ctx.sm_run_steps(6)
    ctx.sync()
    for call in (lambda: ctx.run_steps(1), lambda: ctx.sm_prepare(TOL), lambda: ctx.kinetic_energy(p_end=1),
                 lambda: ctx.det_ratio()):
        with pytest.raises(vm.VmcError) as ei:
            call()
        assert ei.value.status == vm.VMC_ESTATE
    ctx.build_slater()
    with pytest.raises(vm.VmcError) as ei:  # rows rebuilt, factors still of the old rows
        ctx.run_steps(1)
    assert ei.value.status == vm.VMC_ESTATE
    ctx.ilutp(reorder=False)
    pos_mid = ctx.state(0)["pos"]
    log = ctx.run_steps_logged(s.n)
    stats = ctx.stats()[0]
    assert stats["status"] == 0
    rep = replay(s, pos_mid, inst.walkers[0].seed, inst.params.step, _records(log[0]), dec_tol=DEC_TOL)
    _say(f"  sparse steps after standard steps: {rep.summary()}")
    assert rep.pos_mismatch == 0 and rep.sign_mismatch == 0
    assert rep.decision_mismatch_outside_tol == 0
    assert rep.max_dlog < DLOG_TOL
    # a reorder rebuilds the rows itself
    ctx.sm_prepare(TOL)
    ctx.sm_run_steps(3)
    ctx.ilutp(reorder=True)
    ctx.run_steps(3)
    ctx.sync()
    ctx.close()
