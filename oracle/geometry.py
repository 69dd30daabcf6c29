"""Geometry, orbitals and the dense Slater matrix (FP64).

Test infrastructure (see package docstring).

Slater matrix: a_{ij} = phi_j(r_i), rows are particles, columns are orbitals
(Section 2.1, eq. (SlaterMatrix)).  Orbitals are Gaussians centred on lattice
sites (eq. (gaussian)), written with a width sigma_j as exp(-|d|^2/(2 sigma_j^2)),
i.e. k = 1/(2 sigma^2), truncated to zero beyond a cutoff radius (the paper
truncates them too, Section 2.1 and Section 4).  The optional p-like term
p_scale * d_x * exp(-|d|^2/(2 p_sigma^2)) is a second orbital component of one of
the synthetic workloads; it is not in the paper.

Displacements use the minimum image in the periodic box (Section 2.1: particles
are confined to a cube with periodic boundary conditions).  With positions and
sites in [0, L), one conditional shift by L per axis gives the minimum image.
Squared distances are formed as (dx*dx + dy*dy) + dz*dz with every operation a
separate IEEE binary64 rounding (numpy never fuses them), so the sparsity
pattern {d^2 <= rc^2} is bit-reproducible on any IEEE machine that evaluates the
same expression without contraction.
"""
from __future__ import annotations

import numpy as np

from workloads import ORB_GAUSS_PX


def min_image(d: np.ndarray, box) -> np.ndarray:
    """Minimum-image displacement for d in (-L, L): shift by L once if |d| > L/2
    (Section 2.1, periodic cube; reading R8)."""
    box = np.asarray(box, dtype=np.float64)
    half = 0.5 * box
    d = np.where(d > half, d - box, d)
    d = np.where(d < -half, d + box, d)
    return d


def dist2(r: np.ndarray, Z: np.ndarray, box) -> np.ndarray:
    """Squared minimum-image distance between r (...,3) and Z (...,3), summed as
    (dx*dx + dy*dy) + dz*dz (reading R8)."""
    d = min_image(r - Z, box)
    return (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]


def orbital_values(r: np.ndarray, system, cols=None) -> np.ndarray:
    """phi_j(r) for all orbitals j (or the given subset), zero beyond the cutoff:
    the Gaussians of eq. (gaussian), plus the p-like term where the system has it."""
    Z = system.sites if cols is None else system.sites[cols]
    sig = system.sigma if cols is None else system.sigma[cols]
    d = min_image(np.asarray(r, dtype=np.float64)[None, :] - Z, system.box)
    d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    inside = d2 <= system.cutoff * system.cutoff
    val = np.exp(-d2 / (2.0 * sig * sig))
    if system.kind == ORB_GAUSS_PX:
        val = val + system.p_scale * d[:, 0] * np.exp(-d2 / (2.0 * system.p_sigma * system.p_sigma))
    return np.where(inside, val, 0.0)


def row_pattern(r: np.ndarray, system) -> np.ndarray:
    """Sorted orbital ids j with |r - Z_j|^2 <= rc^2 (minimum image): the nonzero
    pattern of a Slater row (Section 2.1, truncated orbitals; reading R8)."""
    d2 = dist2(np.asarray(r, dtype=np.float64)[None, :], system.sites, system.box)
    return np.nonzero(d2 <= system.cutoff * system.cutoff)[0]


def slater_dense(pos: np.ndarray, system, block: int = 256) -> np.ndarray:
    """Dense A[p, j] = phi_j(r_p) in original labels (particles x orbitals),
    eq. (SlaterMatrix)."""
    n = pos.shape[0]
    A = np.zeros((n, system.n), dtype=np.float64)
    for p0 in range(0, n, block):
        p1 = min(n, p0 + block)
        d = min_image(pos[p0:p1, None, :] - system.sites[None, :, :], system.box)
        d2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        inside = d2 <= system.cutoff * system.cutoff
        sg = system.sigma[None, :]
        val = np.exp(-d2 / (2.0 * sg * sg))
        if system.kind == ORB_GAUSS_PX:
            val = val + system.p_scale * d[..., 0] * np.exp(
                -d2 / (2.0 * system.p_sigma * system.p_sigma))
        A[p0:p1] = np.where(inside, val, 0.0)
    return A


def propose(r: np.ndarray, u3, h: float, box) -> np.ndarray:
    """Trial position of one particle: r + h*(2u-1) per axis, wrapped into [0,L)
    by one conditional shift (Section 2.2: move one particle a small random
    distance).  2u-1 is exact for the u01 mapping, so the only roundings are
    the product, the sum and the shift."""
    box = np.asarray(box, dtype=np.float64)
    out = np.empty(3, dtype=np.float64)
    for c in range(3):
        x = float(r[c]) + h * (2.0 * u3[c] - 1.0)
        if x >= box[c]:
            x = x - box[c]
        elif x < 0.0:
            x = x + box[c]
        out[c] = x
    return out
