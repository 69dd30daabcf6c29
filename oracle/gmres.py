"""Right-preconditioned full GMRES with the effective-stability monitor, and the
product-form preconditioner update.  FP64.

Test infrastructure (see package docstring).

GMRES (Saad and Schultz 1986), full (never restarted), solving A M x~ = b with
z = M x~ (Section 3.2, eq. (precondSystem)).  x0 = 0; Arnoldi by modified
Gram-Schmidt; the least-squares problem is reduced by Givens rotations and the
residual norm read off the rotated right-hand side; the iteration stops when
that estimate drops below rtol * ||b|| or after maxit iterations (Section 4:
maxit 40).

Effective stability N = max_i ||v_i - A M v_i||_2 over the Arnoldi vectors of
the solve (eq. (stabilityVecEq)).  Reading: M is the preconditioner the solve
actually uses, i.e. Q (LU)^{-1} followed by the stored rank-one factors.

Preconditioner update (Section 3.2, eqs. (finalMk0), (mkp1), (finalMkm)): after
an accepted move with solution z and ratio 1 + u^T z, the new preconditioner is
(I - zhat u^T) M with zhat = z / (1 + u^T z); with several accepted moves the
factors are applied oldest first after Q (LU)^{-1}.
"""
from __future__ import annotations

import numpy as np

from .ilutp import apply_inverse


class ProductPreconditioner:
    """M = (I - zhat_m u_m^T) ... (I - zhat_1 u_1^T) Q (L U)^{-1}: the ILUTP
    preconditioner kept across accepted moves by eqs. (mkp1) and (finalMkm)."""

    def __init__(self, L, U, q):
        self.L, self.U, self.q = L, U, q
        self.updates = []   # list of (zhat, u) with u dense

    def apply(self, v: np.ndarray) -> np.ndarray:
        """M v: the factors first, then the updates oldest first (eq. (finalMkm))."""
        y = apply_inverse(self.L, self.U, self.q, v)
        for zhat, u in self.updates:
            y = y - zhat * float(u @ y)
        return y

    def add_update(self, z: np.ndarray, u: np.ndarray, ratio: float):
        """After an accepted move: M <- (I - zhat u^T) M with zhat = z / ratio
        (eq. (mkp1))."""
        self.updates.append((z / ratio, u.copy()))


def gmres_right(A, M, b: np.ndarray, rtol: float, maxit: int):
    """Return (z, iters, converged, N, resid_est).

    A: callable or matrix for the product A @ y; M: callable y = M v.
    """
    matvec = A if callable(A) else (lambda y: A @ y)
    n = b.shape[0]
    beta = float(np.linalg.norm(b))
    V = np.zeros((maxit + 1, n))
    Zp = np.zeros((maxit, n))
    H = np.zeros((maxit + 1, maxit))
    cs = np.zeros(maxit)
    sn = np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    V[0] = b / beta
    N = 0.0
    k = 0
    converged = False
    res = beta
    for j in range(maxit):
        Zp[j] = M(V[j])
        w = matvec(Zp[j])
        N = max(N, float(np.linalg.norm(V[j] - w)))
        for i in range(j + 1):
            H[i, j] = float(w @ V[i])
            w = w - H[i, j] * V[i]
        H[j + 1, j] = float(np.linalg.norm(w))
        if H[j + 1, j] != 0.0:
            V[j + 1] = w / H[j + 1, j]
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        den = float(np.hypot(H[j, j], H[j + 1, j]))
        cs[j] = H[j, j] / den
        sn[j] = H[j + 1, j] / den
        H[j, j] = den
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        k = j + 1
        res = abs(g[j + 1])
        if res <= rtol * beta:
            converged = True
            break
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
    z = Zp[:k].T @ y
    return z, k, converged, N, res
