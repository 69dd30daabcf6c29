"""Pins for the oracle's Philox4x64-10 and uniform mapping."""
from fractions import Fraction

import numpy as np

from oracle.rng import philox4x64_10, step_draws, u01


def test_philox_matches_numpy():
    # numpy's Philox advances its counter before producing a block, so a
    # generator started at counter c yields philox(c + 1), philox(c + 2), ...
    for key in [(0, 0), (7, 3), (2**63 + 5, 1), (255, 0)]:
        for c0 in [0, 1, 41, 2**40]:
            bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                                  counter=np.array([c0, 0, 0, 0], dtype=np.uint64))
            raw = [int(x) for x in bg.random_raw(8)]
            assert raw[:4] == list(philox4x64_10((c0 + 1, 0, 0, 0), key))
            assert raw[4:] == list(philox4x64_10((c0 + 2, 0, 0, 0), key))


def test_philox_counter_words_all_used():
    bg = np.random.Philox(key=np.array([5, 9], dtype=np.uint64),
                          counter=np.array([2**64 - 1, 6, 7, 8], dtype=np.uint64))
    raw = [int(x) for x in bg.random_raw(4)]
    # increment carries into word 1
    assert raw == list(philox4x64_10((0, 7, 7, 8), (5, 9)))


def test_u01_exact_and_open_interval():
    for x in [0, 1, 4095, 4096, 2**63, 2**64 - 1, 0x9E3779B97F4A7C15]:
        u = u01(x)
        exact = (Fraction(x >> 12) + Fraction(1, 2)) / Fraction(2**52)
        assert Fraction(u) == exact
        assert 0.0 < u < 1.0
        # 2u - 1 is exact in binary64
        assert Fraction(2.0 * u - 1.0) == 2 * exact - 1


def test_step_draws_distribution():
    us = np.array([step_draws(3, g) for g in range(4000)])
    assert us.shape == (4000, 4)
    assert np.all((us > 0) & (us < 1))
    assert abs(us.mean() - 0.5) < 0.02
    assert abs(us.var() - 1.0 / 12.0) < 0.01
