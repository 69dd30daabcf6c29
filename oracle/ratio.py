"""Determinant ratio of consecutive Slater matrices, by its plain definition.

Test infrastructure (see package docstring).

When particle p moves, row p of A changes by u = a' - a_p (eq. (matrixUpdateU)),
A' = A + e_p u^T (eqs. (MatrixUpdate_1), (matrixUpdate2)), and by the matrix
determinant lemma det(A')/det(A) = 1 + u^T A^{-1} e_p (eqs. (DetRatio),
(detRatioEq)).  The oracle forms z = A^{-1} e_p with a dense LU factorisation
(LAPACK getrf/getrs through scipy; a library primitive) and returns 1 + u^T z.

``StandardAlgorithm`` is the paper's "standard algorithm" (Section 1): keep the
explicit inverse B = A^{-1}, read the ratio off B, update B by Sherman-Morrison
on an accepted move and recompute it from scratch periodically.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg as sla


def ratio_lu(A: np.ndarray, p: int, new_row: np.ndarray):
    """(1 + u^T z, a'^T z) with z = A^{-1} e_p by dense LU with partial pivoting:
    eq. (detRatioEq) with u = a' - a_p, and the same ratio from the new row
    alone (reading R7)."""
    n = A.shape[0]
    lu, piv = sla.lu_factor(A, check_finite=False)
    e = np.zeros(n)
    e[p] = 1.0
    z = sla.lu_solve((lu, piv), e, check_finite=False)
    u = new_row - A[p]
    return 1.0 + float(u @ z), float(new_row @ z)


def det_leibniz(A: np.ndarray) -> float:
    """Determinant by the Leibniz permutation sum (tiny n only): the definition
    of det behind eq. (DetRatio)."""
    n = A.shape[0]
    total = 0.0
    for perm in itertools.permutations(range(n)):
        inv = 0
        for a in range(n):
            for b in range(a + 1, n):
                if perm[a] > perm[b]:
                    inv += 1
        prod = 1.0
        for i in range(n):
            prod *= A[i, perm[i]]
        total += -prod if (inv & 1) else prod
    return total


def ratio_leibniz(A: np.ndarray, p: int, new_row: np.ndarray) -> float:
    """det(A')/det(A) with both determinants by brute force (eq. (DetRatio))."""
    A2 = A.copy()
    A2[p] = new_row
    return det_leibniz(A2) / det_leibniz(A)


class StandardAlgorithm:
    """Explicit inverse + Sherman-Morrison ("standard algorithm", Section 1)."""

    def __init__(self, A: np.ndarray):
        self.A = np.array(A, dtype=np.float64, copy=True)
        self.refresh()

    def refresh(self):
        """B = A^{-1} afresh (the standard algorithm recomputes it from time to
        time to bound the drift of the updates)."""
        self.B = sla.inv(self.A, check_finite=False)

    def ratio(self, p: int, new_row: np.ndarray) -> float:
        """det(A')/det(A) = a'^T A^{-1} e_p (Section 1)."""
        # row p of A' dotted with column p of B
        return float(new_row @ self.B[:, p])

    def accept(self, p: int, new_row: np.ndarray, ratio: float):
        """Row p of A becomes new_row; B follows by Sherman-Morrison (Section 1):
        B <- B - (B e_p)(u^T B) / ratio."""
        u = new_row - self.A[p]
        col = self.B[:, p].copy()
        uB = u @ self.B
        self.B -= np.outer(col, uB / ratio)
        self.A[p] = new_row
