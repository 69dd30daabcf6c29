"""Pins for the oracle's determinant ratio and geometric reorder."""
import os

import numpy as np
import pytest

import workloads as wl
from oracle.chain import free_run
from oracle.geometry import orbital_values, slater_dense
from oracle.ratio import det_leibniz, ratio_leibniz, ratio_lu
from oracle.reorder import geometric_reorder, inverse_perm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n", [3, 5, 6])
def test_ratio_lu_vs_leibniz(n):
    rng = np.random.default_rng(n)
    for _ in range(5):
        A = rng.standard_normal((n, n)) + 2 * np.eye(n)
        p = int(rng.integers(0, n))
        new = rng.standard_normal(n)
        r_lu, r_alt = ratio_lu(A, p, new)
        r_bf = ratio_leibniz(A, p, new)
        assert abs(r_lu - r_bf) <= 1e-12 * max(1.0, abs(r_bf))
        assert abs(r_alt - r_bf) <= 1e-12 * max(1.0, abs(r_bf))
    assert abs(det_leibniz(np.diag([2.0, 3.0, 5.0])) - 30.0) == 0.0


def test_ratio_lu_vs_slogdet_slater():
    inst = wl.plain_n128()
    s = inst.systems[0]
    pos = inst.walkers[0].pos0.copy()
    A = slater_dense(pos, s)
    rng = np.random.default_rng(0)
    for p in [0, 17, 127]:
        rnew = (pos[p] + rng.uniform(-0.25, 0.25, 3)) % s.box
        new = orbital_values(rnew, s)
        A2 = A.copy()
        A2[p] = new
        s1, l1 = np.linalg.slogdet(A)
        s2, l2 = np.linalg.slogdet(A2)
        r, _ = ratio_lu(A, p, new)
        assert np.sign(r) == s1 * s2
        assert abs(np.log(abs(r)) - (l2 - l1)) < 1e-11


def test_ratio_invariants():
    inst = wl.plain_n128()
    s = inst.systems[0]
    pos = inst.walkers[0].pos0.copy()
    A = slater_dense(pos, s)
    p = 9
    # unmoved particle: u = 0 exactly, ratio exactly 1
    r0, _ = ratio_lu(A, p, A[p].copy())
    assert r0 == 1.0
    # back-move after an accepted move gives the reciprocal
    rnew = (pos[p] + np.array([0.2, -0.1, 0.15])) % s.box
    new = orbital_values(rnew, s)
    r1, _ = ratio_lu(A, p, new)
    A2 = A.copy()
    A2[p] = new
    r2, _ = ratio_lu(A2, p, A[p].copy())
    assert abs(r1 * r2 - 1.0) < 1e-12
    # simultaneous row/column permutation leaves the ratio unchanged
    rng = np.random.default_rng(5)
    P = rng.permutation(s.n)
    C = rng.permutation(s.n)
    Ap = A[P][:, C]
    ip = inverse_perm(P)
    r3, _ = ratio_lu(Ap, int(ip[p]), new[C])
    assert abs(r3 - r1) < 1e-12 * abs(r1)


def test_standard_algorithm_matches_fresh_lu():
    inst = wl.plain_n128()
    s = inst.systems[0]
    w = inst.walkers[0]
    recs_lu, pos_lu = free_run(s, w.pos0, w.seed, inst.params.step, 300, mode="lu")
    recs_sm, pos_sm = free_run(s, w.pos0, w.seed, inst.params.step, 300, mode="sm")
    assert [r.accepted for r in recs_lu] == [r.accepted for r in recs_sm]
    for a, b in zip(recs_lu, recs_sm):
        assert abs(np.log(abs(a.ratio)) - np.log(abs(b.ratio))) < 1e-9
    assert np.array_equal(pos_lu, pos_sm)
    acc = np.mean([r.accepted for r in recs_lu])
    assert 0.3 < acc < 0.9


def _line_system():
    return wl.System(lattice=(4, 1, 1), a=1.0, sites=wl.lattice_sites(4, 1, 1),
                     sigma=np.full(4, 0.35), kind=wl.ORB_GAUSS, p_scale=0.0,
                     p_sigma=0.5, cutoff=2.0)


def test_reorder_golden_line4():
    s = _line_system()
    with open(os.path.join(GOLDEN, "reorder_line4.txt")) as f:
        lines = [ln for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(lines) == 3
    for ln in lines:
        xs, row, col = ln.split("|")
        xs = [float(t) for t in xs.split()[1:]]
        pos = np.array([[x, 0.0, 0.0] for x in xs])
        r, c = geometric_reorder(pos, s)
        assert list(r) == [int(t) for t in row.split()]
        assert list(c) == [int(t) for t in col.split()]


def test_reorder_golden_line4_from_start_order():
    """The reorder renumbers the matrix it is given: from a start order other
    than the identity it swaps from there (hand-worked cases D-F, including a
    cascade that changes the matching)."""
    s = _line_system()
    with open(os.path.join(GOLDEN, "reorder_line4_start.txt")) as f:
        lines = [ln for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(lines) == 3
    for ln in lines:
        xs, r0, c0, row, col = ln.split("|")
        xs = [float(t) for t in xs.split()[1:]]
        pos = np.array([[x, 0.0, 0.0] for x in xs])
        r0 = [int(t) for t in r0.split()]
        c0 = [int(t) for t in c0.split()]
        r, c = geometric_reorder(pos, s, r0, c0)
        assert list(r) == [int(t) for t in row.split()]
        assert list(c) == [int(t) for t in col.split()]
        # the start arrays are not modified
        assert r0 == [int(t) for t in ln.split("|")[1].split()]


def test_reorder_start_order_checks():
    s = _line_system()
    pos = np.array([[x, 0.0, 0.0] for x in (0.1, 1.1, 2.1, 3.1)])
    r, c = geometric_reorder(pos, s, np.arange(4), np.arange(4))
    assert np.array_equal(r, np.arange(4)) and np.array_equal(c, np.arange(4))
    with pytest.raises(ValueError):
        geometric_reorder(pos, s, [0, 0, 1, 2], None)


def test_reorder_exact_matching_from_any_start():
    """Particles exactly on distinct orbitals: every start order ends with each
    particle on its own orbital (distance zero on the diagonal)."""
    s = wl.make_system((4, 4, 4), sigma=0.35, cutoff=2.0)
    rng = np.random.default_rng(5)
    pi = rng.permutation(s.n)
    pos = s.sites[pi].copy()
    for t in range(3):
        r0, c0 = rng.permutation(s.n), rng.permutation(s.n)
        row, col = geometric_reorder(pos, s, r0, c0)
        assert np.array_equal(col, pi[row])


def test_reorder_recovers_exact_matching():
    s = wl.make_system((4, 4, 8), sigma=0.35, cutoff=2.0)
    rng = np.random.default_rng(3)
    pi = rng.permutation(s.n)
    pos = s.sites[pi].copy()        # particle p sits exactly on orbital pi[p]
    row, col = geometric_reorder(pos, s)
    assert sorted(row) == list(range(s.n)) and sorted(col) == list(range(s.n))
    # every diagonal pair is at distance zero: orbital col[i] = pi[row[i]]
    assert np.array_equal(col, pi[row])
    A = slater_dense(pos, s)[row][:, col]
    assert np.all(np.diag(A) == 1.0)


def test_reorder_identity_on_own_sites():
    s = wl.make_system((4, 4, 4), cutoff=2.0)
    pos = s.sites + 0.05
    row, col = geometric_reorder(pos, s)
    assert np.array_equal(row, np.arange(s.n)) and np.array_equal(col, np.arange(s.n))
