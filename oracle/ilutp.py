"""Threshold incomplete LU with column pivoting (ILUTP), row-wise, FP64.

Test infrastructure (see package docstring).

The paper preconditions with ILUTP (Saad 1994; Saad's book, Section 10.4): an
incomplete factorisation A Q ~ L U with L unit lower triangular, U upper
triangular and Q a column permutation (Section 3.2, eq. (ilu)); a relative
drop tolerance removes small entries, a limit on extra fill bounds each row of
L and of U, and columns are swapped when the diagonal is small compared with the
largest entry of the row, searching the entire row (Section 4).

Row i is computed as follows (readings of the paper's settings in brackets):

1. w <- row i of A, keyed by original column; tau_i = droptol * ||a_i||_2
   [relative drop tolerance: the 2-norm of the original row], or, with
   norm="mean_abs", droptol * ||a_i||_1 / nnz(a_i), the mean magnitude of the
   row's entries, which is the scale SPARSKIT's ILUT and ILUTP use (Section 4
   names SPARSKIT's ILUTP as the paper's preconditioner);
2. eliminate: repeatedly take the not-yet-visited entry of w whose column sits
   at the smallest position k < i, divide it by U_kk; drop it if its magnitude
   is below tau_i, otherwise store it as l_ik and subtract l_ik times row k of U
   (fill-in is created as needed);
3. drop entries of the U part (positions >= i) below tau_i, never the entry in
   the current diagonal column;
4. keep the nL0 + p largest multipliers in L and the nU0 + p largest
   off-diagonal entries in U, where nL0 / nU0 count row i's original entries
   left / right of the diagonal and p = ceil(nnz(A)/(2n)) [Section 4: extra fill
   of half the average row count, at most doubling nnz]; ties go to the lower
   position;
5. pivot: if permtol * max_j |w_j| > |w_diag| over the kept U part, swap the
   diagonal column with the column of the largest entry (lowest position on
   ties) [Section 4: "entire row"];
6. a zero pivot raises ``SingularPivot``.

U rows are stored with original column labels while the factorisation runs,
because later pivots only exchange positions >= the current row; they are
relabelled to final positions at the end.
"""
from __future__ import annotations

import math

import numpy as np


class SingularPivot(Exception):
    """A zero pivot left after the column pivoting of ILUTP."""


def paper_lfil(nnz: int, n: int) -> int:
    """Extra fill per row allowed in L and in U: half the average row count
    (Section 4's fill rule; reading R14)."""
    return int(math.ceil(nnz / (2.0 * n)))


def ilutp(rows, n: int, droptol: float, permtol: float, lfil: int, norm: str = "l2",
          scales: bool = False):
    """Factor the sparse matrix given as ``rows`` (list of {col: value}).
    ``norm`` selects the drop scale of step 1: "l2" or "mean_abs".  With
    ``scales`` also returns, for every stored entry, the magnitude its value
    was accumulated from (|a_ij| plus the |l_ik u_kj| of every multiplier that
    updated it, including multipliers the fill limit later removed), the scale
    of its rounding error.

    Returns (L, U, q): L[i] = {k: l_ik} strictly lower (positions), U[i] =
    {k: u_ik} upper including the diagonal (positions), q[k] = original column
    at position k, so that (A Q)[i, k] = A[i, q[k]] ~ (L U)[i, k].
    """
    q = list(range(n))
    pos = list(range(n))
    Urows = [None] * n      # original column labels
    Lrows = [None] * n
    Uscale = [None] * n
    Lscale = [None] * n
    for i in range(n):
        a = rows[i]
        if norm == "mean_abs":
            tau = droptol * sum(abs(v) for v in a.values()) / len(a)
        else:
            tau = droptol * math.sqrt(sum(v * v for v in a.values()))
        nL0 = sum(1 for c in a if pos[c] < i)
        nU0 = sum(1 for c in a if pos[c] > i)
        w = dict(a)
        wabs = {c: abs(v) for c, v in a.items()}
        Lrow = {}
        Lsc = {}
        visited = set()
        while True:
            cand = [pos[c] for c in w if pos[c] < i and pos[c] not in visited]
            if not cand:
                break
            k = min(cand)
            visited.add(k)
            c = q[k]
            wk = w.pop(c)
            lik = wk / Urows[k][c]
            sk = wabs.pop(c)
            if abs(lik) < tau:
                continue
            Lrow[k] = lik
            Lsc[k] = (sk + abs(wk) * Uscale[k][c] / abs(Urows[k][c])) / abs(Urows[k][c])
            for c2, v in Urows[k].items():
                if c2 != c:
                    w[c2] = w.get(c2, 0.0) - lik * v
                    wabs[c2] = wabs.get(c2, 0.0) + abs(lik * v) + abs(lik) * Uscale[k][c2]
        # w now holds only columns at positions >= i
        cdiag = q[i]
        off = [(c, v) for c, v in w.items() if c != cdiag and abs(v) >= tau]
        # keep the largest: sort by magnitude descending, then position ascending
        off.sort(key=lambda cv: (-abs(cv[1]), pos[cv[0]]))
        off = off[: nU0 + lfil]
        Lkeep = sorted(Lrow.items(), key=lambda kv: (-abs(kv[1]), kv[0]))[: nL0 + lfil]
        Lrows[i] = dict(Lkeep)
        urow = dict(off)
        if cdiag in w:
            urow[cdiag] = w[cdiag]
        dval = urow.get(cdiag, 0.0)
        best_c, best_v = None, -1.0
        for c, v in urow.items():
            av = abs(v)
            if av > best_v or (av == best_v and pos[c] < pos[best_c]):
                best_c, best_v = c, av
        if best_c is None or best_v == 0.0:
            raise SingularPivot(f"zero pivot at row {i}")
        if permtol * best_v > abs(dval) and best_c != cdiag:
            j = pos[best_c]
            q[i], q[j] = q[j], q[i]
            pos[q[i]] = i
            pos[q[j]] = j
        if urow.get(q[i], 0.0) == 0.0:
            raise SingularPivot(f"zero pivot at row {i}")
        Urows[i] = urow
        Uscale[i] = {c: wabs[c] for c in urow}
        Lscale[i] = {k: Lsc[k] for k in Lrows[i]}
    U = [{pos[c]: v for c, v in Urows[i].items()} for i in range(n)]
    if scales:
        Us = [{pos[c]: v for c, v in Uscale[i].items()} for i in range(n)]
        return Lrows, U, np.array(q), Lscale, Us
    return Lrows, U, np.array(q)


def dense_factors(L, U, n):
    """Dense (L, U) with unit diagonal in L, from the rows ilutp returns
    (eq. (ilu): A Q ~ L U)."""
    Ld = np.eye(n)
    Ud = np.zeros((n, n))
    for i in range(n):
        for k, v in L[i].items():
            Ld[i, k] = v
        for k, v in U[i].items():
            Ud[i, k] = v
    return Ld, Ud


def rows_from_dense(A: np.ndarray):
    """The rows of a dense matrix as {column: value} dicts of its nonzeros."""
    return [{int(j): float(A[i, j]) for j in np.nonzero(A[i])[0]} for i in range(A.shape[0])]


def apply_inverse(L, U, q, v: np.ndarray) -> np.ndarray:
    """y = Q (LU)^{-1} v (eq. (ilu)): forward solve with unit L, backward solve
    with U, then place position c at original column q[c]."""
    n = v.shape[0]
    x = np.array(v, dtype=np.float64, copy=True)
    for i in range(n):
        s = x[i]
        for k, l in L[i].items():
            s -= l * x[k]
        x[i] = s
    for i in range(n - 1, -1, -1):
        s = x[i]
        d = 0.0
        for k, u in U[i].items():
            if k == i:
                d = u
            else:
                s -= u * x[k]
        x[i] = s / d
    y = np.empty(n)
    y[q] = x
    return y
