"""Pins for the oracle's ILUTP, GMRES, effective stability and product-form update."""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle.geometry import orbital_values, slater_dense
from oracle.gmres import ProductPreconditioner, gmres_right
from oracle.ilutp import SingularPivot, dense_factors, ilutp, paper_lfil, rows_from_dense


def _gepp_on_transpose(A):
    """LU with column partial pivoting of A, via LAPACK row pivoting of A^T:
    A^T = P L' U'  =>  A P = (U'^T D^-1)(D L'^T), D = diag(U')."""
    P, Lt, Ut = sla.lu(A.T)
    D = np.diag(Ut)
    Lc = Ut.T / D[None, :]
    Uc = D[:, None] * Lt.T
    q = np.argmax(P, axis=0)   # column k of A P is column q[k] of A
    return Lc, Uc, q


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ilutp_full_fill_is_column_partial_pivoting(seed):
    rng = np.random.default_rng(seed)
    n = 24
    A = rng.standard_normal((n, n))
    L, U, q = ilutp(rows_from_dense(A), n, droptol=0.0, permtol=1.0, lfil=n)
    Ld, Ud = dense_factors(L, U, n)
    Lr, Ur, qr = _gepp_on_transpose(A)
    assert np.array_equal(q, qr)
    assert np.max(np.abs(Ld - Lr)) < 1e-10
    assert np.max(np.abs(Ud - Ur)) < 1e-10 * np.max(np.abs(Ur))
    assert np.linalg.norm(A[:, q] - Ld @ Ud) <= 1e-13 * np.linalg.norm(A) * n


def test_ilutp_no_pivot_and_tridiagonal_exact():
    n = 30
    A = np.diag(np.full(n, 4.0)) + np.diag(np.full(n - 1, -1.0), 1) + np.diag(np.full(n - 1, -2.0), -1)
    L, U, q = ilutp(rows_from_dense(A), n, droptol=0.0, permtol=0.0, lfil=0)
    assert np.array_equal(q, np.arange(n))
    Ld, Ud = dense_factors(L, U, n)
    # a tridiagonal matrix has no fill: ILU(0) is its exact LU (Thomas recurrence)
    d = np.zeros(n)
    d[0] = 4.0
    for i in range(1, n):
        d[i] = 4.0 - (-2.0 / d[i - 1]) * (-1.0)
    assert np.allclose(np.diag(Ud), d, rtol=1e-14, atol=0)
    assert np.allclose(Ld @ Ud, A, atol=1e-13)


def test_ilutp_rules_on_slater_matrix():
    inst = wl.plain_n128()
    s = inst.systems[0]
    A = slater_dense(inst.walkers[0].pos0, s)
    n = s.n
    rows = rows_from_dense(A)
    nnz = sum(len(r) for r in rows)
    p = paper_lfil(nnz, n)
    L, U, q = ilutp(rows, n, droptol=1e-4, permtol=0.1, lfil=p)
    Ld, Ud = dense_factors(L, U, n)
    assert sorted(q) == list(range(n))
    assert np.all(np.triu(Ld, 1) == 0) and np.all(np.diag(Ld) == 1.0)
    assert np.all(np.tril(Ud, -1) == 0) and np.all(np.diag(Ud) != 0)
    rel = np.linalg.norm(A[:, q] - Ld @ Ud) / np.linalg.norm(A)
    assert rel < 1e-3
    for i in range(n):
        tau = 1e-4 * np.linalg.norm(A[i])
        assert all(abs(v) >= tau for k, v in L[i].items())
        assert all(abs(v) >= tau for k, v in U[i].items() if k != i)
        assert len(L[i]) <= len(rows[i]) + p
        assert len(U[i]) - 1 <= len(rows[i]) + p
    assert nnz / n > 20


def test_ilutp_drop_scale_two_norm_and_mean_magnitude():
    # row 1 = (0.5, 10) below U row 0 = (10, 1): its multiplier is 0.05.  With
    # droptol 0.007 the 2-norm scale gives tau = 0.007 * 10.0125 = 0.0701 and
    # drops it (u11 = 10); the mean-magnitude scale gives tau = 0.007 * 5.25 =
    # 0.03675 and keeps it (u11 = 10 - 0.05 * 1 = 9.95).
    A = np.array([[10.0, 1.0], [0.5, 10.0]])
    L, U, q = ilutp(rows_from_dense(A), 2, droptol=0.007, permtol=0.0, lfil=2)
    assert L[1] == {} and U[1] == {1: 10.0}
    L, U, q = ilutp(rows_from_dense(A), 2, droptol=0.007, permtol=0.0, lfil=2, norm="mean_abs")
    assert L[1] == {0: 0.05} and abs(U[1][1] - 9.95) < 1e-15


def test_ilutp_zero_pivot_raises():
    A = np.array([[1.0, 2.0], [2.0, 4.0]])
    with pytest.raises(SingularPivot):
        ilutp(rows_from_dense(A), 2, droptol=0.0, permtol=1.0, lfil=2)


def _setup(droptol=1e-2, permtol=0.1):
    inst = wl.plain_n128()
    s = inst.systems[0]
    pos = inst.walkers[0].pos0.copy()
    A = slater_dense(pos, s)
    rows = rows_from_dense(A)
    nnz = sum(len(r) for r in rows)
    L, U, q = ilutp(rows, s.n, droptol, permtol, paper_lfil(nnz, s.n) if droptol > 0 else s.n)
    return inst, s, pos, A, ProductPreconditioner(L, U, q)


def test_gmres_exact_preconditioner_one_iteration():
    inst, s, pos, A, M = _setup(droptol=0.0, permtol=1.0)
    b = np.zeros(s.n)
    b[7] = 1.0
    z, k, conv, N, res = gmres_right(A, M.apply, b, 1e-10, 40)
    assert conv and k == 1
    assert N < 1e-12
    assert np.linalg.norm(A @ z - b) < 1e-12


def test_gmres_ilu_converges_to_true_residual():
    inst, s, pos, A, M = _setup(droptol=1e-2)
    for i in [0, 50, 127]:
        b = np.zeros(s.n)
        b[i] = 1.0
        z, k, conv, N, res = gmres_right(A, M.apply, b, 1e-10, 40)
        assert conv and k < 40
        assert np.linalg.norm(b - A @ z) < 1e-9
        assert np.allclose(z, np.linalg.solve(A, b), atol=1e-9)


def test_effective_stability_bounds_krylov_vectors():
    # For unit z in K_m(AM, r0): ||(I - AM) z|| <= m N (Section 3.1).
    inst, s, pos, A, M = _setup(droptol=5e-2)
    b = np.zeros(s.n)
    b[3] = 1.0
    z, k, conv, N, res = gmres_right(A, M.apply, b, 1e-14, 6)
    # rebuild the Krylov space of A M from b and test random unit vectors in it
    K = [b / np.linalg.norm(b)]
    for _ in range(k - 1):
        K.append(A @ M.apply(K[-1]))
    Qk, _ = np.linalg.qr(np.array(K).T)
    rng = np.random.default_rng(0)
    for _ in range(20):
        c = rng.standard_normal(Qk.shape[1])
        v = Qk @ c
        v /= np.linalg.norm(v)
        assert np.linalg.norm(v - A @ M.apply(v)) <= k * N * (1 + 1e-9)


def test_update_identity_exact_z():
    # A_{k+1} M_{k+1} = A_k M_k + r u^T M_k / (1 + u^T z), r = e_i - A_k z  (Section 3.2)
    inst, s, pos, A, M = _setup(droptol=1e-2)
    p = 40
    rnew = (pos[p] + np.array([0.1, -0.2, 0.05])) % s.box
    new = orbital_values(rnew, s)
    u = new - A[p]
    e = np.zeros(s.n)
    e[p] = 1.0
    rng = np.random.default_rng(2)
    v = rng.standard_normal(s.n)
    A1 = A.copy()
    A1[p] = new
    # exact z: identity holds with r = 0
    z = np.linalg.solve(A, e)
    ratio = 1 + u @ z
    M1 = ProductPreconditioner(M.L, M.U, M.q)
    M1.add_update(z, u, ratio)
    lhs = A1 @ M1.apply(v)
    rhs = A @ M.apply(v)
    assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(rhs)
    # inexact z: the difference is exactly r u^T M v / (1 + u^T z)
    z2 = z + 1e-4 * rng.standard_normal(s.n)
    r2 = e - A @ z2
    ratio2 = 1 + u @ z2
    M2 = ProductPreconditioner(M.L, M.U, M.q)
    M2.add_update(z2, u, ratio2)
    diff = A1 @ M2.apply(v) - A @ M.apply(v)
    pred = r2 * (u @ M.apply(v)) / ratio2
    assert np.linalg.norm(diff - pred) <= 1e-10 * np.linalg.norm(pred)


def test_stability_study_runs_and_orders_measures():
    """The N1/N2/N study script on a small b.c.c. system: it runs, and with the
    pivoting the paper workload uses the accuracy is good and GMRES converges."""
    import subprocess
    import sys as _sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([_sys.executable, os.path.join(root, "tests", "study_preconditioner_stability.py"),
                          "--K", "4", "--configs", "3"], capture_output=True, text=True, check=True).stdout
    lines = [l for l in out.splitlines() if "N1/|A|" in l]
    assert len(lines) == 3
    for l in lines:
        f = l.split()
        its_max = int(f[2].split("-")[1])
        n1 = float(f[f.index("N1/|A|") + 1])
        assert its_max < 40 and n1 < 0.1
    assert "rank correlation" in out


def test_gmres_is_the_krylov_least_squares_solution():
    """Textbook properties of full GMRES (x0 = 0) on a random nonsymmetric
    system, with M = I: after k iterations z_k minimises ||b - A z|| over
    K_k(A, b) (checked against a least-squares fit on an explicit Krylov
    basis), the Givens estimate equals the true residual, the residuals never
    increase, and at k = n the solve is exact."""
    rng = np.random.default_rng(11)
    n = 10
    A = rng.standard_normal((n, n)) + 3.0 * np.eye(n)
    b = rng.standard_normal(n)
    ident = lambda v: v  # noqa: E731
    prev = np.inf
    for k in range(1, n + 1):
        z, its, conv, N, res = gmres_right(A, ident, b, 0.0, k)
        assert its == k
        true = np.linalg.norm(b - A @ z)
        assert abs(res - true) <= 1e-10 * np.linalg.norm(b)
        assert true <= prev * (1 + 1e-12)
        prev = true
        K = np.empty((n, k))
        K[:, 0] = b / np.linalg.norm(b)
        for j in range(1, k):
            v = A @ K[:, j - 1]
            K[:, j] = v / np.linalg.norm(v)
        c, *_ = np.linalg.lstsq(A @ K, b, rcond=None)
        best = np.linalg.norm(b - A @ (K @ c))
        assert abs(true - best) <= 1e-9 * np.linalg.norm(b)
    assert prev <= 1e-10 * np.linalg.norm(b)


def test_product_preconditioner_keeps_AM_over_several_moves():
    """With exact solves, every accepted move leaves A M unchanged (eq. (mkp1)
    applied repeatedly, eq. (finalMkm)): after three moves of different
    particles A_3 M_3 v = A_0 M_0 v.  Applying the stored factors in the wrong
    order breaks this."""
    inst, s, pos, A0, M0 = _setup(droptol=1e-2)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(s.n)
    target = A0 @ M0.apply(v)
    A = A0.copy()
    M = ProductPreconditioner(M0.L, M0.U, M0.q)
    for p, dr in ((40, (0.1, -0.2, 0.05)), (41, (-0.15, 0.1, 0.2)), (40, (0.05, 0.05, -0.1))):
        rnew = (pos[p] + np.array(dr)) % s.box
        pos[p] = rnew
        new = orbital_values(rnew, s)
        u = new - A[p]
        e = np.zeros(s.n)
        e[p] = 1.0
        z = np.linalg.solve(A, e)   # the exact solve
        ratio = 1.0 + u @ z
        M.add_update(z, u, ratio)
        A[p] = new
    got = A @ M.apply(v)
    assert np.linalg.norm(got - target) <= 1e-10 * np.linalg.norm(target)
    # the same updates in reverse order do not keep the product
    R = ProductPreconditioner(M0.L, M0.U, M0.q)
    R.updates = list(reversed(M.updates))
    assert np.linalg.norm(A @ R.apply(v) - target) > 1e-6 * np.linalg.norm(target)
