"""Seeded synthetic inputs for the sparse determinant-ratio VMC workloads.

This module only generates input data: lattice sites, orbital widths, initial
particle positions, per-walker seeds and the solver parameters of each named
workload. It contains none of the method's arithmetic (no orbital evaluation,
no Slater matrix, no ratio, no solver).  Both the CPU oracle and the GPU path
consume what it returns.

Lattice convention: ``Lx x Ly x Lz`` cubic cells of side ``a`` in a periodic
box ``(Lx*a, Ly*a, Lz*a)``, each holding ``nb`` sites at the fractional offsets
``basis[b]`` (one site at the corner for simple cubic; the corner and the body
centre for b.c.c.).  Site ``j = b + nb*(ix + Lx*(iy + Ly*iz))`` sits at
``((ix, iy, iz) + basis[b])*a``.  Particle ``p`` starts at site ``p`` plus a
jitter and is wrapped into ``[0, L)`` per axis.

The paper's own workload is Gaussian orbitals exp(-k|d|^2), k = 1, on a b.c.c.
lattice of cube side 2.031 with n = 2K^3 (Section 2.1, eq. (gaussian);
Section 4): ``paper_bcc`` below.  The other named workloads use a simple-cubic
lattice with a geometric cutoff instead.  All are synthetic in the same way the
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

SC_BASIS = ((0.0, 0.0, 0.0),)
BCC_BASIS = ((0.0, 0.0, 0.0), (0.5, 0.5, 0.5))

SETUP_STREAM = 1   # Philox key word 1 used for per-walker set-up draws
SYSTEM_STREAM = 2  # Philox key word 1 used for shared-system draws


@dataclasses.dataclass
class System:
    """One physical system: orbital centres and orbital shapes."""
    lattice: tuple            # (Lx, Ly, Lz) cell counts
    a: float                  # cell side
    sites: np.ndarray         # (n, 3) float64, wrapped into [0, L)
    sigma: np.ndarray         # (n,) float64 Gaussian widths per orbital
    kind: int                 # ORB_GAUSS or ORB_GAUSS_PX
    p_scale: float
    p_sigma: float
    cutoff: float
    basis: tuple = SC_BASIS   # fractional site offsets within a cell

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
        Lx, Ly, Lz = self.lattice
        nominal = lattice_sites(Lx, Ly, Lz, self.a, self.basis)
        d = self.sites - nominal
        box = self.box
        d = d - box * np.round(d / box)
        return float(np.max(np.abs(d))) if self.n else 0.0


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
    refine_tol: float = 1e-10     # refinement stop: ||r|| <= tol * min(1,|ratio|)
    refine_maxit: int = 4
    sweeps: int = 1
    ilu_work_cap: int = 0         # ILUTP work-row capacity (0: the library default)
    ilu_drop_norm: int = 0        # ILUTP drop scale: 0 = row 2-norm, 1 = mean magnitude
    plain_stop: bool = False      # ratio solves stop at the tolerance itself (no ratio-relative target)


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


def lattice_sites(Lx: int, Ly: int, Lz: int, a: float = 1.0, basis=SC_BASIS) -> np.ndarray:
    nb = len(basis)
    j = np.arange(Lx * Ly * Lz * nb)
    cell = j // nb
    frac = np.stack([(cell % Lx), (cell // Lx) % Ly, cell // (Lx * Ly)], axis=1).astype(np.float64)
    frac = frac + np.asarray(basis, dtype=np.float64)[j % nb]
    return frac * a


def wrap(x: np.ndarray, box: np.ndarray) -> np.ndarray:
    """Conditional single-shift wrap into [0, L) (inputs lie within one box of it)."""
    x = np.where(x >= box, x - box, x)
    x = np.where(x < 0.0, x + box, x)
    return x


def initial_positions(sites: np.ndarray, box: np.ndarray, seed: int, jitter: float,
                      gen: Optional[np.random.Generator] = None, normal: bool = False) -> np.ndarray:
    """Sites plus a jitter: uniform on [-jitter, jitter]^3, or normal with
    standard deviation ``jitter`` per axis (wrapped, so it may exceed a box)."""
    g = gen if gen is not None else _gen(seed, SETUP_STREAM)
    if normal:
        d = g.normal(0.0, jitter, size=sites.shape)
        x = np.mod(sites + d, box)
        return np.where(x >= box, x - box, x)
    d = g.uniform(-jitter, jitter, size=sites.shape)
    return wrap(sites + d, box)


def make_system(lattice, a=1.0, sigma=0.35, kind=ORB_GAUSS, p_scale=0.0, p_sigma=0.5,
                cutoff=2.0, site_jitter_sd=0.0, sigma_lognormal_sd=0.0, seed=0,
                basis=SC_BASIS) -> System:
    Lx, Ly, Lz = lattice
    sites = lattice_sites(Lx, Ly, Lz, a, basis)
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
                  kind=kind, p_scale=p_scale, p_sigma=p_sigma, cutoff=cutoff,
                  basis=tuple(tuple(float(x) for x in b) for b in basis))


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


PAPER_BCC_A = 2.031          # cube side (Section 4)
PAPER_K = 1.0                # Gaussian decay rate k of eq. (gaussian)
PAPER_DROP = 1e-5            # entries below 1e-5 * max|a_ij| are dropped (Section 4)


def paper_bcc(K: int = 7, n_walkers: int = 64, step: float = 0.55, sweeps: int = 120,
              permtol: float = 0.05) -> Instance:
    """The paper's experiment (Section 4): n = 2K^3 electrons, Gaussian orbitals
    exp(-k|d|^2) with k = 1 on a b.c.c. lattice of K^3 cubes of side 2.031,
    entries below 1e-5 times the largest dropped, ILUTP droptol 0.01 and
    permtol 0.05 (swap columns when 0.05 times the row's largest entry exceeds
    the diagonal), GMRES rtol 1e-6 and at most 40 iterations, reorder when
    N > 100 or the iterations reach four times their average, 120 sweeps, FP64.

    The pivot threshold 0.05 gives stable factorisations because each reorder
    starts from the order the previous one left (Section 3.1 renumbers the
    matrix as it stands): on equilibrated configurations at n = 686, fresh
    factorisations then need 5-9 iterations with N below 10 and keep about 53
    entries per row in L and U together (the paper: 8.9 iterations, 55.0).
    Starting every reorder from particle and orbital ids instead leaves about one
    row in ten with a diagonal twenty times below the row's largest entry, and
    the same factorisations need 13-30 iterations with N up to 1e5.

    Ratio solves stop at rtol itself, the paper's criterion, so that the
    iteration counts compare with its Table "cost" (the library's default goes
    on to rtol * min(1, |ratio|)).

    Readings: the drop tolerance scales each row's mean magnitude, as in
    SPARSKIT's ILUTP, which the paper uses; the largest entry is taken as 1 (an
    orbital at its own centre),
    so the drop rule is the geometric cutoff |d|^2 <= ln(1e5)/k; the proposal
    half-width (not given) is chosen so the acceptance is near the paper's
    0.588; start positions are the sites plus uniform jitter in [-0.3, 0.3]
    per axis, as for the other workloads (the first 20 sweeps, which the
    paper discards, equilibrate the chain).
    With droptol 0.01 a row's elimination visits up to about 12-16 K^2
    entries before the fill limit applies, hence the ILUTP work capacity
    20 K^2 (it fits the LDS of one workgroup up to K = 12)."""
    sigma = 1.0 / np.sqrt(2.0 * PAPER_K)
    cutoff = float(np.sqrt(np.log(1.0 / PAPER_DROP) / PAPER_K))
    s = make_system((K, K, K), a=PAPER_BCC_A, sigma=sigma, cutoff=cutoff, basis=BCC_BASIS)
    ws = [Walker(0, initial_positions(s.sites, s.box, w, 0.3), w) for w in range(n_walkers)]
    return Instance("paper_bcc_n%d" % s.n, [s], ws,
                    Params(step=step, sweeps=sweeps, droptol=0.01, permtol=permtol, gmres_rtol=1e-6,
                           gmres_maxit=40, n_thresh=100.0, iter_factor=4.0, mixed=False,
                           ilu_work_cap=20 * K * K, ilu_drop_norm=1, plain_stop=True))


WORKLOADS = {
    "plain_n128": plain_n128,
    "fp64_n1024": fp64_n1024,
    "uneven_batch": uneven_batch,
    "mixed_n4000": mixed_n4000,
    "stress_n8192": stress_n8192,
    "paper_bcc": paper_bcc,
}
