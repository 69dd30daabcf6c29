"""Geometric greedy reordering of particles (rows) and orbitals (columns).

Test infrastructure (see package docstring).

Section 3.1 gives the algorithm: label particles and orbitals 1..n; for each
position i except the last, find among the orbitals still at positions i..n the
one closest to the particle at position i; if it is not already at position i,
swap the two columns; otherwise find among the particles at positions i..n the
one closest to the orbital at position i and, if it is not the one at position
i, swap the two rows.

Readings where the paper is silent:
- the labelling starts from the identity (particle ids, orbital ids) on every
  reorder, so the result is a function of the positions alone;
- "closest" is the smallest squared minimum-image distance between the particle
  and the orbital centre, evaluated as in ``geometry.dist2``;
- ties go to the first position in the current order (numpy.argmin returns the
  first minimum).
"""
from __future__ import annotations

import numpy as np

from .geometry import dist2


def geometric_reorder(pos: np.ndarray, system):
    """Return (row, col): row[i] = particle at row position i, col[i] = orbital at
    column position i."""
    n = pos.shape[0]
    row = np.arange(n)
    col = np.arange(n)
    Z = system.sites
    for i in range(n - 1):
        d2 = dist2(pos[row[i]][None, :], Z[col[i:]], system.box)
        j = i + int(np.argmin(d2))
        if j != i:
            col[i], col[j] = col[j], col[i]
        else:
            d2p = dist2(pos[row[i:]], Z[col[i]][None, :], system.box)
            k = i + int(np.argmin(d2p))
            if k != i:
                row[i], row[k] = row[k], row[i]
    return row, col


def inverse_perm(perm: np.ndarray) -> np.ndarray:
    """inv[perm[i]] = i: from position-to-label to label-to-position."""
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.shape[0])
    return inv
