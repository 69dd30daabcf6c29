"""Pins for the oracle's geometry, orbitals and dense Slater matrix."""
from fractions import Fraction

import numpy as np

import workloads as wl
from oracle.geometry import dist2, min_image, orbital_values, propose, row_pattern, slater_dense


def _brute_min_d2(r, Z, box):
    best = np.inf
    for sx in (-1, 0, 1):
        for sy in (-1, 0, 1):
            for sz in (-1, 0, 1):
                d = r - (Z + np.array([sx, sy, sz]) * box)
                best = min(best, float(d @ d))
    return best


def test_min_image_equals_nearest_periodic_image():
    rng = np.random.default_rng(1)
    box = np.array([4.0, 5.0, 8.0])
    for _ in range(300):
        r = rng.uniform(0, 1, 3) * box
        Z = rng.uniform(0, 1, 3) * box
        d = min_image(r - Z, box)
        assert np.all(np.abs(d) <= 0.5 * box)
        assert abs(float(dist2(r[None], Z[None], box)[0]) - _brute_min_d2(r, Z, box)) < 1e-12


def test_site_centred_neighbour_counts():
    # points of Z^3 within radius rc of the origin: shells 0,1,sqrt2,sqrt3,2 give
    # 1+6+12+8+6 = 33 for rc = 2; adding sqrt5 (24) and sqrt6 (24) gives 81 for rc = 2.5
    s = wl.make_system((8, 8, 16), cutoff=2.0)
    for site in [0, 77, 1023]:
        assert len(row_pattern(s.sites[site], s)) == 33
    s25 = wl.make_system((10, 20, 20), cutoff=2.5)
    for site in [0, 1234, 3999]:
        assert len(row_pattern(s25.sites[site], s25)) == 81


def test_orbital_closed_forms():
    s = wl.make_system((8, 8, 8), sigma=0.35, cutoff=2.0)
    v = orbital_values(s.sites[0], s)
    assert v[0] == 1.0
    assert abs(v[1] - np.exp(-1.0 / (2 * 0.35**2))) < 1e-15
    # periodic neighbour across the x boundary (site 7 sits at x = 7 = -1 mod 8)
    assert abs(v[7] - np.exp(-1.0 / (2 * 0.35**2))) < 1e-15
    assert v[3] == 0.0  # distance 3 > cutoff
    px = wl.make_system((8, 8, 8), sigma=0.35, kind=wl.ORB_GAUSS_PX, p_scale=0.1,
                        p_sigma=0.5, cutoff=2.5)
    r = np.array([1.0, 0.0, 0.0])
    v = orbital_values(r, px)
    # site 0 at origin: d = (1,0,0): gauss + 0.1 * 1 * exp(-1/(2*0.25))
    assert abs(v[0] - (np.exp(-1 / (2 * 0.35**2)) + 0.1 * np.exp(-2.0))) < 1e-15
    # site 2 at x=2: d = (-1,0,0): the p-term changes sign
    assert abs(v[2] - (np.exp(-1 / (2 * 0.35**2)) - 0.1 * np.exp(-2.0))) < 1e-15


def test_slater_symmetric_on_sites_and_pattern():
    s = wl.make_system((4, 4, 8), sigma=0.35, cutoff=2.0)
    A = slater_dense(s.sites.copy(), s)
    assert np.array_equal(A, A.T)
    assert np.all(np.diag(A) == 1.0)
    inst = wl.plain_n128()
    pos = inst.walkers[0].pos0
    A = slater_dense(pos, s)
    for p in [0, 5, 127]:
        assert np.array_equal(np.nonzero(A[p])[0], row_pattern(pos[p], s))
        assert np.allclose(A[p], orbital_values(pos[p], s), rtol=0, atol=0)


def test_propose_exact_arithmetic():
    box = np.array([4.0, 4.0, 8.0])
    r = np.array([0.01, 3.99, 5.5])
    u = (0.1, 0.9, 0.5)
    out = propose(r, u, 0.25, box)
    for c in range(3):
        x = Fraction(float(r[c])) + Fraction(float(0.25 * (2.0 * u[c] - 1.0)))
        x = float(x)  # one rounding of the sum (the product is exact-rounded separately)
        if x >= box[c]:
            x -= box[c]
        elif x < 0:
            x += box[c]
        assert out[c] == x
        assert 0.0 <= out[c] < box[c]


def test_paper_bcc_lattice_matches_section4():
    """Section 4: cube side 2.031, nearest-neighbour distance 1.759, density
    3/(4 pi) = 0.2387 electrons per unit volume, n = 2 K^3; entries below 1e-5
    of the largest (1) are dropped."""
    from oracle.geometry import dist2
    for K in (4, 7):
        s = wl.paper_bcc(K=K, n_walkers=1).systems[0]
        assert s.n == 2 * K ** 3
        vol = float(np.prod(s.box))
        assert abs(s.n / vol - 3.0 / (4.0 * np.pi)) < 5e-5
        d = np.sqrt(dist2(s.sites[0][None, :], s.sites[1:], s.box))
        assert abs(d.min() - 1.759) < 5e-4
        assert np.sum(np.abs(d - d.min()) < 1e-12) == 8          # b.c.c. coordination
        k = 1.0 / (2.0 * s.sigma[0] ** 2)
        assert abs(k - 1.0) < 1e-15
        assert abs(np.exp(-k * s.cutoff ** 2) - 1e-5) < 1e-18
