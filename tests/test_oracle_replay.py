"""The replay checker that the GPU parity tests rely on, pinned on the CPU.

A log from the oracle's own free run replays with no error; mistakes planted
in a copy of that log (a ratio off by a relative 1e-8, a wrong sign, a moved
particle put elsewhere, a decision flipped far from or within the decision
tolerance, a record of the wrong particle) are each caught and counted in the
right class.  Section 2.2 fixes what a step is: one particle moved, accepted
when ratio^2 exceeds the uniform draw.
"""
import dataclasses

import numpy as np

import workloads as wl
from oracle.chain import ReplayReport, free_run, positions_after, replay


def _run(steps=96, mode="lu"):
    inst = wl.small_instance((2, 2, 4))
    s = inst.systems[0]
    w = inst.walkers[0]
    recs, pos = free_run(s, w.pos0, w.seed, inst.params.step, steps, mode=mode)
    return inst, s, w, recs, pos


def _replay(inst, s, w, recs, **kw):
    return replay(s, w.pos0, w.seed, inst.params.step, recs, **kw)


def test_own_log_replays_clean():
    inst, s, w, recs, pos = _run()
    for mode in ("lu", "sm"):
        rep = _replay(inst, s, w, recs, mode=mode)
        assert rep.steps == len(recs)
        assert rep.pos_mismatch == rep.sign_mismatch == rep.decision_mismatch == 0
        assert rep.max_dlog < 1e-12
    assert np.array_equal(positions_after(w.pos0, recs), pos)
    assert "p99.9" in rep.summary() and f"{len(recs)} steps" in rep.summary()


def test_planted_ratio_error_is_measured():
    inst, s, w, recs, _ = _run()
    k = 17
    bad = list(recs)
    bad[k] = dataclasses.replace(recs[k], ratio=recs[k].ratio * (1.0 + 1e-8))
    rep = _replay(inst, s, w, bad)
    assert abs(rep.max_dlog - 1e-8) < 1e-11
    assert int(np.argmax(rep.dlogs)) == k
    assert rep.decision_mismatch == 0 and rep.pos_mismatch == 0


def test_planted_sign_and_position_errors_are_counted():
    # each mistake sits in the last record of a truncated log, so nothing
    # after it depends on how the replay handles it
    inst, s, w, recs, _ = _run()
    bad = recs[:6]
    bad[5] = dataclasses.replace(recs[5], ratio=-recs[5].ratio)
    rep = _replay(inst, s, w, bad)
    assert rep.sign_mismatch == 1 and rep.pos_mismatch == 0 and rep.decision_mismatch == 0
    bad = recs[:10]
    bad[9] = dataclasses.replace(recs[9], new_pos=np.asarray(recs[9].new_pos) + np.array([1e-12, 0.0, 0.0]))
    rep = _replay(inst, s, w, bad)
    assert rep.pos_mismatch == 1 and rep.sign_mismatch == 0
    bad = recs[:13]
    bad[12] = dataclasses.replace(recs[12], particle=(recs[12].particle + 1) % s.n)
    rep = _replay(inst, s, w, bad)
    assert rep.pos_mismatch == 1


def test_flipped_decisions_classified_by_tolerance():
    inst, s, w, recs, _ = _run()
    gap = [abs(r.ratio * r.ratio - r.u_acc) for r in recs]
    for k in (int(np.argmax(gap)), int(np.argmin(gap))):
        bad = recs[:k + 1]
        bad[k] = dataclasses.replace(recs[k], accepted=not recs[k].accepted)
        # a tolerance wider than the step's gap: a mismatch, but inside it
        rep = _replay(inst, s, w, bad, dec_tol=2.0 * gap[k])
        assert rep.decision_mismatch == 1 and rep.decision_mismatch_outside_tol == 0
        # a narrower one: outside it
        rep = _replay(inst, s, w, bad, dec_tol=0.5 * gap[k])
        assert rep.decision_mismatch == 1 and rep.decision_mismatch_outside_tol == 1


def test_empty_log():
    inst, s, w, _, _ = _run(steps=1)
    rep = _replay(inst, s, w, [])
    assert rep == ReplayReport()
    assert rep.summary().startswith("0 steps")


def test_replay_in_pieces_matches_whole():
    """The pooled replay cut into pieces (each from the positions its log
    gives, with a fresh inverse) agrees with the replay of the whole log."""
    import sys
    sys.path.insert(0, __file__.rsplit("/", 1)[0])
    from _replay_pool import replay_walkers
    inst = wl.fp64_n1024(1)
    s = inst.system_of(0)
    w = inst.walkers[0]
    log, _ = free_run(s, w.pos0, w.seed, inst.params.step, 90, mode="sm")
    recs = np.zeros(len(log), dtype=[("step", "i8"), ("particle", "i4"), ("new_pos", "f8", 3), ("ratio", "f8"),
                                     ("u_acc", "f8"), ("flags", "i4")])
    for k, r in enumerate(log):
        recs[k] = (r.g, r.particle, r.new_pos, r.ratio, r.u_acc, int(r.accepted))
    whole = replay_walkers("fp64_n1024", inst.params.step, {0: w.pos0}, {0: recs}, 1)[0]
    pieces = replay_walkers("fp64_n1024", inst.params.step, {0: w.pos0}, {0: recs}, 3, parts=3)[0]
    assert pieces.steps == whole.steps == len(log)
    assert pieces.pos_mismatch == whole.pos_mismatch == 0
    assert pieces.decision_mismatch == whole.decision_mismatch == 0
    np.testing.assert_allclose(pieces.oracle_ratios, whole.oracle_ratios, rtol=1e-11)
    assert pieces.max_dlog < 1e-11
