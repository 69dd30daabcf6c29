"""The ILUTP runs with its fast configuration (eight rows in flight, small
tables); when a row overflows those tables, the full one (four rows, larger
tables) resumes at the first unfinished row for a window of rows, then the
fast one takes over again.  The row algorithm is the same in
both (Section 3.2, eq. (ilu)), so the factors must agree bit for bit with a
factorisation that uses the full configuration alone (a given ilu_work_cap),
both when the fast tables hold every row and when a test knob shrinks them so
that the factorisation falls back again and again."""
import numpy as np
import pytest

import paper_1008_5113_amd as vm
import workloads as wl

pytestmark = pytest.mark.gpu


def _factors(inst, walkers, **kw):
    ctx = vm.Context.from_instance(inst, walkers=walkers, **kw)
    try:
        ctx.ilutp(reorder=True)
        ctx.sync()
        retries = sum(s["ilu_retries"] for s in ctx.stats())
        return [ctx.state(w, factors=True) for w in range(len(walkers))], retries
    finally:
        ctx.close()


def _same(a, b, what):
    for key in ("l_len", "u_len", "ilu_perm", "col_site", "row_particle", "a_len"):
        np.testing.assert_array_equal(a[key], b[key], err_msg=f"{what}: {key}")
    np.testing.assert_array_equal(a["u_diag"].view(np.int64), b["u_diag"].view(np.int64), err_msg=f"{what}: u_diag")
    for r in range(len(a["l_len"])):
        ll, ul = a["l_len"][r], a["u_len"][r]
        for key, m in (("l_col", ll), ("u_col", ul)):
            np.testing.assert_array_equal(a[key][r, :m], b[key][r, :m], err_msg=f"{what}: {key} row {r}")
        for key, m in (("l_val", ll), ("u_val", ul)):
            np.testing.assert_array_equal(a[key][r, :m].view(np.int64), b[key][r, :m].view(np.int64),
                                          err_msg=f"{what}: {key} row {r}")


@pytest.mark.parametrize("case", ["mixed_n4000", "uneven_batch", "stress_n8192"])
def test_fast_and_full_configurations_give_the_same_factors(case):
    if case == "mixed_n4000":
        inst, ws = wl.mixed_n4000(4), [0, 1, 2, 3]
    elif case == "uneven_batch":
        inst, ws = wl.uneven_batch(8), list(range(8))
    else:
        inst, ws = wl.stress_n8192(1), [0]
    print(f"ilutp configurations: {case}, walkers {ws}", flush=True)
    full, r_full = _factors(inst, ws, ilu_work_cap=512)
    fast, r_fast = _factors(inst, ws)
    retried, r_small = _factors(inst, ws, test_knobs=vm.vmcdet.TEST_ILU_FAST_SMALL)
    print(f"  fallback windows: full alone {r_full}, fast {r_fast}, small fast tables {r_small}", flush=True)
    assert r_full == 0
    # a row of A alone (63 or more entries here) nearly fills 64-entry tables,
    # so the fill of the first rows overflows them
    assert r_small > 0
    for w in range(len(ws)):
        assert full[w]["l_len"].sum() > 0
        _same(full[w], fast[w], f"{case} walker {ws[w]} fast")
        _same(full[w], retried[w], f"{case} walker {ws[w]} retried")
