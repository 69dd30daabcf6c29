"""bench.py's algorithmic byte count (the roofline's `achieved`), checked on the
CPU against the per-step formula written out by hand for known counts."""
import bench


def _stats(iters, inner, solves, passes, msum):
    return {"iters": iters, "inner_solves": inner, "solves": solves, "refine_passes": passes,
            "update_sum": msum}


def test_fp64_path_bytes():
    n, nA, nL, nU = 100, 700, 150, 250
    s0 = [_stats(0, 0, 0, 0, 0)]
    s1 = [_stats(30, 10, 10, 0, 50)]          # 10 solves of 3 iterations, 5 stored updates on average
    per_iter = (700 + 150 + 250) * (8 + 2) + 100 * 8 * (1 + 5) + 4 * 100 * 8
    want = 30 * per_iter + 10 * 100 * 8
    assert bench.algorithmic_bytes(s0, s1, (nA, nL, nU), n, mixed=False) == want


def test_mixed_path_bytes_and_walker_sum():
    n, nA, nL, nU = 100, 700, 150, 250
    s0 = [_stats(5, 2, 1, 1, 0), _stats(0, 0, 0, 0, 0)]
    # walker 0: 40 iterations in 20 inner solves (10 ratio solves, 10
    # refinement passes), 60 stored updates per inner solve on average
    s1 = [_stats(45, 22, 11, 11, 1200), _stats(4, 2, 1, 1, 0)]
    def walker(iters, inner, solves, passes, msum):
        m = msum / inner
        per_iter = (700 + 150 + 250) * (4 + 2) + 100 * 4 * (1 + m) + 4 * 100 * 4
        return iters * per_iter + inner * 800 + (solves + passes) * (700 * 10 + 16 * 100)
    want = walker(40, 20, 10, 10, 1200) + walker(4, 2, 1, 1, 0)
    got = bench.algorithmic_bytes(s0, s1, (nA, nL, nU), n, mixed=True)
    assert abs(got - want) <= 1e-9 * want
