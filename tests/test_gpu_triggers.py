"""The reorder triggers of Section 4 (N above its threshold, a solve that misses
its tolerance within the iteration limit, iterations at a multiple of their
running average), the walker that stays unconverged after the reorder
(VMC_ENOCONV), the refusal of a forced acceptance of a zero ratio, and the
device-pointer mode of the per-move calls, all through the C-ABI.  Where a
chain runs, every step is replayed by the dense-LU oracle."""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle.chain import StepRecord, replay

pytestmark = pytest.mark.gpu

DLOG_TOL = 1e-10
DEC_TOL = 1e-9


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


def _records(log_row):
    return [StepRecord(int(r["step"]), int(r["particle"]), np.array(r["new_pos"]), float(r["ratio"]),
                       float(r["u_acc"]), bool(r["flags"] & 1)) for r in log_row]


def _replay_ok(inst, log_row):
    s = inst.systems[0]
    w = inst.walkers[0]
    rep = replay(s, w.pos0, w.seed, inst.params.step, _records(log_row))
    _say("  replay: " + rep.summary())
    assert rep.pos_mismatch == 0
    assert rep.decision_mismatch_outside_tol == 0
    assert rep.max_dlog <= DLOG_TOL, rep.max_dlog
    return rep


def _check_record_fields(vm, log_row, precision):
    # ln|ratio| as the device computed it, to the last few ulps of numpy's
    assert np.all(np.abs(log_row["log_abs_ratio"] - np.log(np.abs(log_row["ratio"]))) <= 1e-14)
    assert np.all(log_row["inner_solves"] == 1 + log_row["refinements"])
    if precision == vm.PREC_FP64:
        assert np.all(log_row["refinements"] == 0)


@pytest.mark.parametrize("precision", [0, 1])
def test_trigger_n_threshold(vm, precision):
    """n_thresh = 0: N > 0 at every solve, so every step reorders, refactors and
    solves again, with the N trigger named in its record."""
    _say(f"case: N-threshold trigger, precision={precision}")
    inst = wl.plain_n128()
    ctx = vm.Context.from_instance(inst, precision=precision, n_thresh=0.0)
    ctx.ilutp(reorder=True)
    log = ctx.run_steps_logged(64)[0]
    st = ctx.stats()[0]
    ctx.close()
    assert np.all(log["flags"] & vm.FLAG_REORDERED) and np.all(log["flags"] & vm.FLAG_TRIG_N)
    assert np.all(log["flags"] & vm.FLAG_CONVERGED) and not np.any(log["flags"] & vm.FLAG_NOCONV)
    assert st["reorders"] == 64 + 1 and st["status"] == 0
    _check_record_fields(vm, log, precision)
    _replay_ok(inst, log)


@pytest.mark.parametrize("precision", [0, 1])
def test_trigger_not_converged(vm, precision):
    """The first solve of each step is capped at one iteration (test knob), so
    it misses its tolerance: the not-converged trigger reorders, refactors and
    solves again without the cap, and the ratios still meet the target."""
    _say(f"case: not-converged trigger, precision={precision}")
    inst = wl.small_instance(lattice=(4, 4, 8), droptol=1e-2)
    ctx = vm.Context.from_instance(inst, precision=precision, test_knobs=vm.vmcdet.TEST_FIRST_SOLVE_ONE_ITER)
    ctx.ilutp(reorder=True)
    log = ctx.run_steps_logged(48)[0]
    ctx.close()
    trig = (log["flags"] & vm.FLAG_TRIG_NOCONV) != 0
    assert trig.sum() >= 40, trig.sum()
    assert np.all(log["flags"][trig] & vm.FLAG_REORDERED)
    assert np.all(log["flags"] & vm.FLAG_CONVERGED) and not np.any(log["flags"] & vm.FLAG_NOCONV)
    _check_record_fields(vm, log, precision)
    _replay_ok(inst, log)


@pytest.mark.parametrize("precision", [0, 1])
def test_trigger_iterations_over_average(vm, precision):
    """iter_factor 1 after 5 solves: a solve needing at least the running
    average of iterations reorders; the records name the trigger."""
    _say(f"case: iteration-average trigger, precision={precision}")
    inst = wl.plain_n128()
    ctx = vm.Context.from_instance(inst, precision=precision, iter_factor=1.0, iter_min_solves=5)
    ctx.ilutp(reorder=True)
    log = ctx.run_steps_logged(96)[0]
    ctx.close()
    trig = (log["flags"] & vm.FLAG_TRIG_ITERS) != 0
    assert trig.sum() >= 5, trig.sum()
    assert not np.any(trig[:5])          # the average is used only after 5 solves
    assert np.all(log["flags"][trig] & vm.FLAG_REORDERED)
    assert np.all(log["flags"] & vm.FLAG_CONVERGED)
    _check_record_fields(vm, log, precision)
    _replay_ok(inst, log)


@pytest.mark.parametrize("precision", [0, 1])
def test_noconv_after_reorder_stops_walker(vm, precision):
    """gmres_maxit = 1 with a loose factorisation: the solve misses its
    tolerance before and after the reorder, so the walker stops with
    VMC_ENOCONV (per-move call and persistent run alike); a refactor clears it."""
    _say(f"case: unconverged after reorder, precision={precision}")
    inst = wl.small_instance(lattice=(4, 4, 8), n_walkers=2, droptol=1e-2)
    ctx = vm.Context.from_instance(inst, precision=precision, gmres_maxit=1, refine_maxit=1)
    ctx.ilutp(reorder=True)
    ratio, info = ctx.det_ratio(walkers=[0], check=False)
    f = int(info["flags"][0])
    assert f & vm.FLAG_NOCONV and f & vm.FLAG_TRIG_NOCONV and f & vm.FLAG_REORDERED
    assert not (f & vm.FLAG_CONVERGED)
    with pytest.raises(vm.VmcError) as ei:
        ctx.sync()
    assert ei.value.status == vm.VMC_ENOCONV
    # no move is pending and the walker refuses further steps
    with pytest.raises(vm.VmcError) as ei:
        ctx.accept(walkers=[0])
    assert ei.value.status == vm.VMC_ESTATE
    assert ctx.stats()[0]["status"] == vm.VMC_ENOCONV
    # the persistent path stops the other walker the same way
    ctx.run_steps(5)
    with pytest.raises(vm.VmcError) as ei:
        ctx.sync()
    assert ei.value.status == vm.VMC_ENOCONV
    st = ctx.stats()
    assert st[1]["status"] == vm.VMC_ENOCONV and st[1]["steps"] == 0
    # a refactor clears the status
    ctx.ilutp(reorder=True)
    assert all(s["status"] == 0 for s in ctx.stats())
    ctx.close()


def test_forced_accept_of_zero_ratio_is_refused(vm):
    """A pending ratio of exactly 0 (test knob): a forced acceptance returns
    VMC_ESINGULAR and leaves the move pending; rejecting it then succeeds, the
    Metropolis rule never accepts it, and the positions never change."""
    _say("case: forced accept of a zero ratio")
    inst = wl.small_instance(lattice=(4, 4, 4), n_walkers=2)
    ctx = vm.Context.from_instance(inst, test_knobs=vm.vmcdet.TEST_ZERO_RATIO)
    ctx.ilutp(reorder=True)
    pos0 = [ctx.state(w)["pos"].copy() for w in range(2)]
    r, _ = ctx.det_ratio()
    assert np.all(r == 0.0)
    with pytest.raises(vm.VmcError) as ei:
        ctx.accept(walkers=[0, 1], decisions=[1, 0])
    assert ei.value.status == vm.VMC_ESINGULAR
    # walker 1's rejection went through; walker 0's move is still pending
    with pytest.raises(vm.VmcError) as ei:
        ctx.accept(walkers=[1], decisions=[0])
    assert ei.value.status == vm.VMC_ESTATE
    assert not ctx.accept(walkers=[0], decisions=[0])[0]
    r, _ = ctx.det_ratio()
    assert not np.any(ctx.accept())          # Metropolis: 0 > u never holds
    for w in range(2):
        assert np.array_equal(ctx.state(w)["pos"], pos0[w])
    ctx.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_device_pointer_mode_matches_host_mode(vm, precision):
    """The per-move calls with device arrays (vmc_params.device_ptrs) give the
    same ratios, records and decisions as with host arrays, bit for bit, and
    report a forced zero-ratio acceptance at vmc_sync."""
    import torch
    _say(f"case: device-pointer mode, precision={precision}")
    inst = wl.small_instance(lattice=(4, 4, 4), n_walkers=3)
    host = vm.Context.from_instance(inst, precision=precision)
    dev = vm.Context.from_instance(inst, precision=precision, device_ptrs=1)
    for c in (host, dev):
        c.ilutp(reorder=True)
    nw = 3
    ratio_d = torch.zeros(nw, dtype=torch.float64, device="cuda")
    info_d = torch.zeros(nw * vm.STEP_RECORD_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    acc_d = torch.zeros(nw, dtype=torch.uint8, device="cuda")
    for k in range(30):
        rh, ih = host.det_ratio()
        ah = host.accept()
        torch.cuda.synchronize()
        dev.det_ratio_device(ratio_d.data_ptr(), info_d.data_ptr())
        dev.accept_device(None, acc_d.data_ptr())
        dev.sync()
        rd = ratio_d.cpu().numpy()
        idev = info_d.cpu().numpy().view(vm.STEP_RECORD_DTYPE)
        assert np.array_equal(rh, rd), k
        assert np.array_equal(ih["ratio"], idev["ratio"]) and np.array_equal(ih["flags"], idev["flags"])
        assert np.array_equal(ah, acc_d.cpu().numpy().astype(bool)), k
    host.close()
    dev.close()
    # caller errors surface at vmc_sync in this mode
    z = vm.Context.from_instance(inst, precision=precision, device_ptrs=1,
                                 test_knobs=vm.vmcdet.TEST_ZERO_RATIO)
    z.ilutp(reorder=True)
    z.det_ratio_device(ratio_d.data_ptr())
    ones = torch.ones(nw, dtype=torch.uint8, device="cuda")
    z.accept_device(ones.data_ptr(), acc_d.data_ptr())
    with pytest.raises(vm.VmcError) as ei:
        z.sync()
    assert ei.value.status == vm.VMC_ESINGULAR
    z.sync()                                  # reported once, then cleared
    # walker lists are refused in this mode
    with pytest.raises(vm.VmcError):
        z.det_ratio(walkers=[0])
    z.close()
