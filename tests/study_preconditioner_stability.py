"""Accuracy N1, stability N2 and effective stability N of the paper's ILUTP
(Section 3.1, eqs. (accuracyEq), (stabilityEq), (stabilityVecEq)) against
GMRES iterations, on the oracle.  A study, not a test (pytest does not
collect it):

    python tests/study_preconditioner_stability.py --K 7 --permtol 0.05 --configs 16

Configurations come from the oracle's chain on the paper's b.c.c. system,
every n/2 steps after --burnin sweeps (default 20, the sweeps the paper
discards; --burnin 0 studies the equilibration itself).  Each configuration is
reordered starting from the previous configuration's order, as the path does
(the first from the identity); --identity-start starts every reorder from the
identity instead.  Each is reordered and factored afresh (droptol 0.01 on the
mean-magnitude scale, the fill rule of the workloads); for it the study prints
N1/||A||_F = ||AQ - LU||_F / ||A||_F, N2 = ||I - AQ (LU)^{-1}||_F, and, over six
solves A z = e_i by right-preconditioned GMRES to 1e-6, the largest N and the
iteration counts; at the end the rank correlations of the iterations with
each measure.
"""
import argparse
import os
import sys

import numpy as np
from scipy.stats import spearmanr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
import oracle.ilutp as oi  # noqa: E402
from oracle.chain import free_run  # noqa: E402
from oracle.geometry import slater_dense  # noqa: E402
from oracle.gmres import gmres_right  # noqa: E402
from oracle.reorder import geometric_reorder  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--K", type=int, default=7)
    ap.add_argument("--permtol", type=float, default=0.05)
    ap.add_argument("--configs", type=int, default=16)
    ap.add_argument("--burnin", type=int, default=20)
    ap.add_argument("--identity-start", action="store_true")
    a = ap.parse_args()
    inst = wl.paper_bcc(K=a.K, n_walkers=1, permtol=a.permtol)
    s = inst.systems[0]
    n = s.n
    pos = inst.walkers[0].pos0.copy()
    start = 0
    if a.burnin:
        _, pos = free_run(s, pos, inst.walkers[0].seed, inst.params.step, a.burnin * n, mode="sm")
        start = a.burnin * n
    rng = np.random.default_rng(1)
    out = []
    row = col = None
    for c in range(a.configs):
        _, pos = free_run(s, pos, inst.walkers[0].seed, inst.params.step, n // 2,
                          start_step=start + c * (n // 2), mode="sm")
        A = slater_dense(pos, s)
        if a.identity_start:
            row = col = None
        row, col = geometric_reorder(pos, s, row, col)
        Ar = A[row][:, col]
        rows = oi.rows_from_dense(Ar)
        nnz = sum(len(r) for r in rows)
        L, U, q = oi.ilutp(rows, n, inst.params.droptol, a.permtol, oi.paper_lfil(nnz, n), norm="mean_abs")
        Ld, Ud = oi.dense_factors(L, U, n)
        AQ = Ar[:, q]
        n1 = np.linalg.norm(AQ - Ld @ Ud) / np.linalg.norm(AQ)
        n2 = np.linalg.norm(np.eye(n) - AQ @ np.linalg.inv(Ld @ Ud))
        its, Ns = [], []
        for i in rng.choice(n, 6, replace=False):
            b = np.zeros(n)
            b[i] = 1.0
            _, k, conv, N, _ = gmres_right(Ar, lambda v: oi.apply_inverse(L, U, q, v), b, 1e-6, 40)
            its.append(k if conv else 41)
            Ns.append(N)
        fill = (sum(len(x) for x in L) + sum(len(x) for x in U)) / n
        out.append((max(its), max(Ns), n1, n2))
        print(f"{c:3d}  iterations {min(its)}-{max(its)}  N {max(Ns):.2e}  N1/|A| {n1:.2e}  N2 {n2:.2e}  "
              f"nnz(L+U)/n {fill:.1f}", flush=True)
    R = np.array(out)
    print("rank correlation with the iterations: N %.2f, N2 %.2f, N1 %.2f"
          % (spearmanr(R[:, 0], R[:, 1])[0], spearmanr(R[:, 0], R[:, 3])[0], spearmanr(R[:, 0], R[:, 2])[0]))


if __name__ == "__main__":
    main()
