"""Philox4x64-10 counter-based RNG and the per-step draws of the Metropolis chain.

Test infrastructure (see package docstring).

Philox4x64 is defined in Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC'11): a 4-word counter and a 2-word key; each of
the 10 rounds multiplies two counter words by fixed odd constants, splits the
128-bit products into high and low halves, mixes the high halves with the other
two counter words and the key by XOR, and permutes; the key is advanced by two
Weyl constants between rounds.  Pinned against ``numpy.random.Philox``.

The paper leaves the random-number stream of the chain unspecified (Section 2.2
only asks for a uniform draw on (0,1) per step).  Reading used here: walker seed
``s`` gives the key ``(s, 0)``; step ``g`` (0-based count of steps the walker has
made) uses counter ``(g, 0, 0, 0)``; the four output words give the three
proposal displacements and the acceptance uniform, in that order.
"""
from __future__ import annotations

MASK64 = (1 << 64) - 1
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B

TWO_M52 = 2.0 ** -52


def philox4x64_10(counter, key):
    """Return the 4 output words for a 4-word counter and a 2-word key."""
    c0, c1, c2, c3 = (int(x) & MASK64 for x in counter)
    k0, k1 = (int(x) & MASK64 for x in key)
    for _ in range(10):
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + PHILOX_W0) & MASK64
        k1 = (k1 + PHILOX_W1) & MASK64
    return (c0, c1, c2, c3)


def u01(x: int) -> float:
    """Map a 64-bit word to a double in (0,1): the top 52 bits plus one half,
    scaled by 2^-52 (reading R1).  Every step is exact in binary64, so the value
    is the same on any IEEE machine; it never equals 0 or 1."""
    return (float(x >> 12) + 0.5) * TWO_M52


def step_draws(seed: int, g: int):
    """(u_x, u_y, u_z, u_acc) for walker seed ``seed`` at step ``g``: the move and
    the acceptance draw of one Metropolis step (Section 2.2; reading R1)."""
    w = philox4x64_10((g, 0, 0, 0), (seed, 0))
    return tuple(u01(x) for x in w)
