"""Geometric greedy reordering of particles (rows) and orbitals (columns).

Test infrastructure (see package docstring).

Section 3.1 gives the algorithm: label particles and orbitals 1..n; for each
position i except the last, find among the orbitals still at positions i..n the
one closest to the particle at position i; if it is not already at position i,
swap the two columns; otherwise find among the particles at positions i..n the
one closest to the orbital at position i and, if it is not the one at position
i, swap the two rows.

Readings where the paper is silent:
- the labelling the algorithm starts from is the matrix's current order: the
  result of the previous reorder (without the column pivots of the
  factorisation that followed it), and the identity (particle ids, orbital
  ids) before the first one.  Starting every reorder from the identity instead
  leaves the last positions of the greedy pass with far-away orbitals (a
  diagonal twenty or more times below the row's largest entry in about one row
  in ten of the paper's equilibrated b.c.c. matrices), which the pivot
  threshold of Section 4 does not repair;
- "closest" is the smallest squared minimum-image distance between the particle
  and the orbital centre, evaluated as in ``geometry.dist2``;
- ties go to the first position in the current order (numpy.argmin returns the
  first minimum).
"""
from __future__ import annotations

import numpy as np

from .geometry import dist2


def geometric_reorder(pos: np.ndarray, system, row=None, col=None):
    """Return (row, col): row[i] = particle at row position i, col[i] = orbital at
    column position i.  ``row`` and ``col`` give the order to start from (the
    previous reorder's result; the identity when omitted)."""
    n = pos.shape[0]
    row = np.arange(n) if row is None else np.array(row, dtype=np.int64, copy=True)
    col = np.arange(n) if col is None else np.array(col, dtype=np.int64, copy=True)
    if sorted(row.tolist()) != list(range(n)) or sorted(col.tolist()) != list(range(n)):
        raise ValueError("the start order must be two permutations of 0..n-1")
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
