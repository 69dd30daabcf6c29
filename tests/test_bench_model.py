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


def test_driver_command_line_parses_and_plans_equal_launches():
    # the exact argument list the round-end benchmark uses
    args = bench.parse_args(["--gpus", "1", "--steps", "20", "--warmup", "5"])
    assert (args.gpus, args.steps, args.warmup, args.block) == (1, 20, 5, bench.BLOCK)
    assert args.m_max == 200 and args.autotune == 1
    plan = bench.launch_plan(args.steps, args.warmup, args.block, bool(args.autotune))
    roles = [r for r, _ in plan]
    assert roles.count("autotune") == 1 and roles.count("warmup") == 5 and roles.count("timed") == 20
    assert roles[-1] == "logged"
    # every launch of the step kernel has the same size, so a profiler's
    # per-launch average is the timed launches' duration
    assert {s for _, s in plan} == {args.block}


def test_any_steps_and_warmup_are_accepted():
    for steps, warmup in [(1, 0), (3, 7), (20, 5), (7, 13)]:
        args = bench.parse_args(["--steps", str(steps), "--warmup", str(warmup), "--block", "50"])
        plan = bench.launch_plan(args.steps, args.warmup, args.block, False)
        assert sum(1 for r, _ in plan if r == "timed") == steps
        assert sum(1 for r, _ in plan if r == "warmup") == warmup


def test_defaults_are_the_driver_shape():
    args = bench.parse_args([])
    assert (args.steps, args.warmup) == (bench.STEPS, bench.WARMUP)
    assert args.cpu_procs == 0   # the host's cores, capped


def test_bad_counts_are_refused():
    import pytest
    for argv in (["--steps", "0"], ["--warmup", "-1"], ["--block", "0"]):
        with pytest.raises(SystemExit):
            bench.parse_args(argv)


def test_uneven_sizes_sum_per_walker():
    """Walkers of different n (the uneven batch): the count is the sum of each
    walker's own count with its own n and factor sizes."""
    s0 = [_stats(0, 0, 0, 0, 0), _stats(0, 0, 0, 0, 0)]
    s1 = [_stats(30, 10, 10, 0, 50), _stats(12, 4, 4, 0, 8)]
    sizes = [(100, (700, 150, 250)), (432, (3000, 700, 900))]
    want = sum(bench.algorithmic_bytes([a], [b], nnz, n, mixed=False)
               for a, b, (n, nnz) in zip(s0, s1, sizes))
    got = bench.algorithmic_bytes(s0, s1, [nnz for _, nnz in sizes], [n for n, _ in sizes], mixed=False)
    assert got == want
