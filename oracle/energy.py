"""Kinetic energy of the Slater-determinant wave function, exact (FP64).

Test infrastructure (see package docstring).

Section 2.3 (Local Energy): the local energy needs, for every particle p, the
Laplacian of Psi with respect to r_p divided by Psi.  Replacing row p of the
Slater matrix by the Laplacians of the orbitals at r_p turns this into one more
determinant ratio, lap_p^T A^{-1} e_p (the matrix determinant lemma of
eq. (detRatioEq) with the whole row replaced).  Section 4, eq. (energyEq),
samples the kinetic energy per particle at the end of every sweep, with
hbar = m = 1:

    E = (1/n) sum_p t_p,   t_p = -(1/2) sum_j lap phi_j(r_p) (A^{-1})_{jp}.

Reading (index order of eq. (energyEq)): with a_{pj} = phi_j(r_p) as in
eq. (SlaterMatrix), the Laplacian of orbital j at particle p multiplies
(A^{-1})_{jp}; for the paper's Gaussians exp(-k|d|^2) the factor
-(1/2) lap phi / phi is (1/2)(6k - 4k^2 |d|^2), which is eq. (energyEq) with the
particle and orbital indices of its distance and of A read consistently.

The oracle forms A^{-1} e_p by a dense LU factorisation (LAPACK through scipy,
a library primitive).  Orbitals are truncated at the cutoff exactly as in
``geometry``; the Laplacian of the truncated function is taken inside the
cutoff sphere only (the jump at the sphere, of relative size
exp(-rc^2/(2 sigma^2)), is ignored, as the paper ignores dropped entries).

Laplacians, with c = 1/sigma^2 and e = 1/p_sigma^2 (derived by differentiating
the orbital definitions of ``geometry``):
  Gaussian exp(-|d|^2 c/2):            (c^2 |d|^2 - 3c) * exp(-|d|^2 c/2)
  p-like term s d_x exp(-|d|^2 e/2):   s d_x (e^2 |d|^2 - 5e) exp(-|d|^2 e/2)
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from workloads import ORB_GAUSS_PX

from .geometry import min_image, slater_dense


def _lap_from_disp(d: np.ndarray, sig: np.ndarray, system) -> np.ndarray:
    d2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    inside = d2 <= system.cutoff * system.cutoff
    c = 1.0 / (sig * sig)
    lap = (c * c * d2 - 3.0 * c) * np.exp(-0.5 * c * d2)
    if system.kind == ORB_GAUSS_PX:
        e = 1.0 / (system.p_sigma * system.p_sigma)
        lap = lap + system.p_scale * d[..., 0] * (e * e * d2 - 5.0 * e) * np.exp(-0.5 * e * d2)
    return np.where(inside, lap, 0.0)


def laplacian_values(r: np.ndarray, system) -> np.ndarray:
    """lap phi_j(r) for all orbitals j (zero beyond the cutoff): the Laplacian of
    eq. (gaussian)'s orbitals in closed form, as eq. (energyEq) needs it."""
    d = min_image(np.asarray(r, dtype=np.float64)[None, :] - system.sites, system.box)
    return _lap_from_disp(d, system.sigma, system)


def laplacian_dense(pos: np.ndarray, system) -> np.ndarray:
    """Dense Lap[p, j] = lap phi_j(r_p) in original labels (eq. (energyEq))."""
    d = min_image(np.asarray(pos, dtype=np.float64)[:, None, :] - system.sites[None, :, :], system.box)
    return _lap_from_disp(d, system.sigma[None, :], system)


def kinetic_terms(pos: np.ndarray, system, particles=None) -> np.ndarray:
    """t_p = -(1/2) lap_p^T A^{-1} e_p for the given particles (all by default):
    particle p's term of eq. (energyEq) (reading R22), by dense LU."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    ps = np.arange(n) if particles is None else np.asarray(particles, dtype=np.int64)
    A = slater_dense(pos, system)
    lu = sla.lu_factor(A, check_finite=False)
    E = np.zeros((n, ps.size))
    E[ps, np.arange(ps.size)] = 1.0
    Zc = sla.lu_solve(lu, E, check_finite=False)          # columns A^{-1} e_p
    lap = laplacian_dense(pos[ps], system)                 # rows lap_p
    return -0.5 * np.einsum("kj,jk->k", lap, Zc)


def kinetic_energy(pos: np.ndarray, system) -> float:
    """Kinetic energy per particle, eq. (energyEq)."""
    return float(np.mean(kinetic_terms(pos, system)))
