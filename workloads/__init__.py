"""Seeded synthetic inputs for the sparse determinant-ratio VMC workloads.

This module only generates input data: lattice sites, orbital widths, initial
particle positions, per-walker seeds and the solver parameters of each named
workload. It contains none of the method's arithmetic (no orbital evaluation,
no Slater matrix, no ratio, no solver).  Both the CPU oracle and the GPU path
consume what it returns.

Lattice convention: a simple-cubic lattice of ``Lx x Ly x Lz`` sites with
spacing ``a``; site ``j = ix + Lx*(iy + Ly*iz)`` sits at ``(ix, iy, iz)*a`` in a
periodic box ``(Lx*a, Ly*a, Lz*a)``.  Particle ``p`` starts at site ``p`` plus a
uniform jitter and is wrapped into ``[0, L)`` per axis.

The paper's own workload is Gaussian orbitals on a b.c.c. lattice (Section 2.1,
eq. (gaussian); Section 4).  The named workloads below use a simple-cubic
lattice with a geometric cutoff instead, and are synthetic in the same way the
paper's are: there is no dataset behind them.

All transcendental set-up draws (Gaussian site jitter, lognormal widths) are
made here once, on the host, with numpy's Philox generator in a dedicated
stream, and shipped as data to both implementations.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

ORB_GAUSS = 0      # phi_j(r) = exp(-|d|^2 / (2 sigma_j^2))
ORB_GAUSS_PX = 1   # Gaussian plus p_scale * d_x * exp(-|d|^2 / (2 p_sigma^2))

SETUP_STREAM = 1   # Philox key word 1 used for per-walker set-up draws
SYSTEM_STREAM = 2  # Philox key word 1 used for shared-system draws


@dataclasses.dataclass
class System:
    """One physical system: orbital centres and orbital shapes."""
    lattice: tuple            # (Lx, Ly, Lz) site counts
    a: float                  # lattice spacing
    sites: np.ndarray         # (n, 3) float64, wrapped into [0, L)
    sigma: np.ndarray         # (n,) float64 Gaussian widths per orbital
    kind: int                 # ORB_GAUSS or ORB_GAUSS_PX
    p_scale: float
    p_sigma: float
    cutoff: float

    @property
    def n(self) -> int:
        return int(self.sites.shape[0])

    @property
    def box(self) -> np.ndarray:
        return np.array([self.lattice[0] * self.a, self.lattice[1] * self.a,
                         self.lattice[2] * self.a], dtype=np.float64)

    def site_margin(self) -> float:
        """Largest per-axis deviation of a site from its nominal lattice point
        (minimum image), so a lattice-neighbourhood search can be widened."""
        n = self.n
        Lx, Ly, _ = self.lattice
        j = np.arange(n)
        nominal = np.stack([(j % Lx), (j // Lx) % Ly, j // (Lx * Ly)], axis=1) * self.a
        d = self.sites - nominal
        box = self.box
        d = d - box * np.round(d / box)
        return float(np.max(np.abs(d))) if n else 0.0


@dataclasses.dataclass
class Walker:
    system: int               # index into Instance.systems
    pos0: np.ndarray          # (n, 3) float64 initial positions in [0, L)
    seed: int                 # Philox key word 0 for this walker's moves


@dataclasses.dataclass
class Params:
    """Solver and chain parameters (readings of the paper's settings)."""
    step: float = 0.25            # proposal half-width h
    droptol: float = 1e-4         # ILUTP relative drop tolerance
    permtol: float = 0.1          # ILUTP pivot tolerance
    lfil: int = -1                # -1: extra fill per row = ceil(nnz(A)/(2n))
    gmres_rtol: float = 1e-10     # GMRES relative residual tolerance
    gmres_maxit: int = 40         # full GMRES, no restart
    n_thresh: float = 100.0       # effective-stability reorder threshold
    iter_factor: float = 4.0      # reorder when iterations >= factor * average
    iter_min_solves: int = 10     # solves before the average is trusted
    m_max: int = 32               # stored rank-one updates before a refactor
    mixed: bool = False           # FP32 Krylov / factors, FP64 refinement
    inner_rtol: float = 1e-6      # inner FP32 solve tolerance (mixed)
    refine_tol: float = 1e-11     # refinement stop: ||r|| <= tol * min(1,|ratio|)
    refine_maxit: int = 4
    sweeps: int = 1


@dataclasses.dataclass
class Instance:
    name: str
    systems: List[System]
    walkers: List[Walker]
    params: Params

    def system_of(self, w: int) -> System:
        return self.systems[self.walkers[w].system]


def _gen(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=np.array([seed, stream], dtype=np.uint64)))


def lattice_sites(Lx: int, Ly: int, Lz: int, a: float = 1.0) -> np.ndarray:
    j = np.arange(Lx * Ly * Lz)
    return np.stack([(j % Lx), (j // Lx) % Ly, j // (Lx * Ly)], axis=1).astype(np.float64) * a


def wrap(x: np.ndarray, box: np.ndarray) -> np.ndarray:
    """Conditional single-shift wrap into [0, L) (inputs lie within one box of it)."""
    x = np.where(x >= box, x - box, x)
    x = np.where(x < 0.0, x + box, x)
    return x


def initial_positions(sites: np.ndarray, box: np.ndarray, seed: int, jitter: float,
                      gen: Optional[np.random.Generator] = None) -> np.ndarray:
    g = gen if gen is not None else _gen(seed, SETUP_STREAM)
    d = g.uniform(-jitter, jitter, size=sites.shape)
    return wrap(sites + d, box)


def make_system(lattice, a=1.0, sigma=0.35, kind=ORB_GAUSS, p_scale=0.0, p_sigma=0.5,
                cutoff=2.0, site_jitter_sd=0.0, sigma_lognormal_sd=0.0, seed=0) -> System:
    Lx, Ly, Lz = lattice
    sites = lattice_sites(Lx, Ly, Lz, a)
    n = sites.shape[0]
    box = np.array([Lx * a, Ly * a, Lz * a])
    g = _gen(seed, SYSTEM_STREAM)
    if site_jitter_sd > 0.0:
        sites = wrap(sites + g.normal(0.0, site_jitter_sd, size=sites.shape), box)
    if sigma_lognormal_sd > 0.0:
        sig = sigma * np.exp(sigma_lognormal_sd * g.standard_normal(n))
    else:
        sig = np.full(n, float(sigma))
    return System(lattice=(Lx, Ly, Lz), a=a, sites=sites, sigma=sig.astype(np.float64),
                  kind=kind, p_scale=p_scale, p_sigma=p_sigma, cutoff=cutoff)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def plain_n128() -> Instance:
    """n=128 electrons on a 4x4x8 sc lattice, Gaussian width 0.35, cutoff 2.0,
    jitter U[-0.3,0.3]^3, proposal half-width 0.25, 20 sweeps, FP64, seed 0."""
    s = make_system((4, 4, 8), sigma=0.35, cutoff=2.0)
    w = [Walker(0, initial_positions(s.sites, s.box, 0, 0.3), 0)]
    return Instance("plain_n128", [s], w, Params(step=0.25, sweeps=20, droptol=1e-4,
                                                 permtol=0.1, gmres_rtol=1e-10))


def fp64_n1024(n_walkers: int = 256) -> Instance:
    """n=1024 on an 8x8x16 lattice, 256 walkers (seeds 0..255), 50 sweeps, ILUTP
    droptol 1e-4, permtol 0.1, GMRES rtol 1e-10, FP64."""
    s = make_system((8, 8, 16), sigma=0.35, cutoff=2.0)
    ws = [Walker(0, initial_positions(s.sites, s.box, w, 0.3), w) for w in range(n_walkers)]
    return Instance("fp64_n1024", [s], ws, Params(step=0.25, sweeps=50, droptol=1e-4,
                                                  permtol=0.1, gmres_rtol=1e-10))


UNEVEN_LATTICES = [(6, 6, 12), (8, 8, 16), (10, 10, 20), (12, 12, 24)]


def uneven_batch(n_walkers: int = 2048) -> Instance:
    """Walkers of uneven size: n drawn uniformly from {432, 1024, 2000, 3456},
    per-walker Gaussian width U[0.3,0.4], cutoff 2.0, FP64, 20 sweeps."""
    systems, walkers = [], []
    for w in range(n_walkers):
        g = _gen(w, SETUP_STREAM)
        lat = UNEVEN_LATTICES[int(g.integers(0, 4))]
        sig = float(g.uniform(0.3, 0.4))
        s = make_system(lat, sigma=sig, cutoff=2.0)
        systems.append(s)
        walkers.append(Walker(len(systems) - 1, initial_positions(s.sites, s.box, w, 0.3, gen=g), w))
    return Instance("uneven_batch", systems, walkers, Params(step=0.25, sweeps=20))


def mixed_n4000(n_walkers: int = 512) -> Instance:
    """n=4000 on a 10x20x20 lattice, 512 walkers; Gaussian width 0.35 plus a
    p-like term 0.1*d_x*exp(-|d|^2/(2*0.5^2)), cutoff 2.5, 30 sweeps; FP32
    Krylov, factors and SpMV with FP64 refinement, ratio and monitor."""
    s = make_system((10, 20, 20), sigma=0.35, kind=ORB_GAUSS_PX, p_scale=0.1,
                    p_sigma=0.5, cutoff=2.5)
    ws = [Walker(0, initial_positions(s.sites, s.box, w, 0.3), w) for w in range(n_walkers)]
    # m_max: the refactor period balancing the measured ILUTP cost against the
    # growing cost of applying the stored updates
    return Instance("mixed_n4000", [s], ws, Params(step=0.25, sweeps=30, mixed=True, m_max=96))


def stress_n8192(n_walkers: int = 64) -> Instance:
    """n=8192 on a 16x16x32 lattice with sites jittered by N(0,0.1^2), lognormal
    widths (median 0.35, sigma 0.15), cutoff 2.5, proposal half-width 0.4, 64
    walkers, mixed precision, 20 sweeps."""
    s = make_system((16, 16, 32), sigma=0.35, kind=ORB_GAUSS, cutoff=2.5,
                    site_jitter_sd=0.1, sigma_lognormal_sd=0.15, seed=0)
    ws = [Walker(0, initial_positions(s.sites, s.box, w, 0.3), w) for w in range(n_walkers)]
    return Instance("stress_n8192", [s], ws, Params(step=0.4, sweeps=20, mixed=True))


def small_instance(lattice=(4, 4, 4), n_walkers=1, sigma=0.35, cutoff=2.0, kind=ORB_GAUSS,
                   p_scale=0.0, step=0.25, jitter=0.3, seed0=0, **pkw) -> Instance:
    """A small instance for tests (any lattice, any walker count)."""
    s = make_system(lattice, sigma=sigma, kind=kind, p_scale=p_scale, cutoff=cutoff)
    ws = [Walker(0, initial_positions(s.sites, s.box, seed0 + w, jitter), seed0 + w)
          for w in range(n_walkers)]
    return Instance("small", [s], ws, Params(step=step, **pkw))


WORKLOADS = {
    "plain_n128": plain_n128,
    "fp64_n1024": fp64_n1024,
    "uneven_batch": uneven_batch,
    "mixed_n4000": mixed_n4000,
    "stress_n8192": stress_n8192,
}
