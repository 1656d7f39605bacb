"""Checks of the seeded input generators against their closed forms."""

import math

import numpy as np
import pytest
from scipy import stats

import workloads


def test_plummer_mass_profile():
    """Cumulative mass M(<r) = r^3/(r^2+a^2)^{3/2} with a = 3 pi/16 (NB units)."""
    c = workloads.make_cluster(20000, 1, imf=False)
    r = np.linalg.norm(c.pos, axis=0)
    a = 3 * math.pi / 16
    cdf = lambda x: np.minimum((x ** 3 / (x * x + a * a) ** 1.5) / workloads.PLUMMER_MASS_CUT, 1.0)
    assert stats.kstest(r, cdf).pvalue > 1e-3


def test_plummer_virial_equilibrium(orc):
    """Equal masses: 2T/|U| ~ 1 and E ~ -1/4 in Henon units."""
    c = workloads.make_cluster(4000, 2, imf=False)
    _, phi = orc.force_newton(c.pos, c.mass)
    U = 0.5 * np.dot(c.mass, phi)
    T = 0.5 * np.dot(c.mass, (c.vel ** 2).sum(axis=0))
    assert 2 * T / abs(U) == pytest.approx(1.0, abs=0.08)
    assert T + U == pytest.approx(-0.25, abs=0.02)


def test_kroupa_slopes():
    rng = np.random.default_rng(3)
    m = workloads.kroupa_imf(rng, 400000, m_max=150.0)
    assert m.min() >= 0.08 and m.max() <= 150.0
    for lo, hi, alpha in ((0.1, 0.4, 1.3), (1.0, 20.0, 2.3)):
        edges = np.logspace(math.log10(lo), math.log10(hi), 12)
        h, _ = np.histogram(m, bins=edges)
        dn_dm = h / np.diff(edges)
        mid = np.sqrt(edges[1:] * edges[:-1])
        slope = np.polyfit(np.log(mid), np.log(dn_dm), 1)[0]
        assert slope == pytest.approx(-alpha, abs=0.08)


def test_binaries_fraction_and_orbits():
    n = 20000
    c = workloads.make_cluster(n, 4, imf=True, binary_fraction=0.5)
    assert c.n_binaries == 5000
    assert c.mass.sum() == pytest.approx(1.0, rel=1e-12)
    # nearest neighbour of each binary member is its companion at < 2 a_max
    from scipy.spatial import cKDTree
    d, _ = cKDTree(c.pos.T).query(c.pos.T, k=2)
    close = (d[:, 1] < 2e-2).sum()
    assert close >= 2 * c.n_binaries * 0.99


def test_binary_orbit_elements():
    """Kepler solution: recover a (log-uniform range) and thermal e from (dr, dv)."""
    rng = np.random.default_rng(5)
    nb = 20000
    mt = np.full(nb, 1e-3)
    a = np.exp(rng.uniform(math.log(1e-5), math.log(1e-2), nb))
    e = np.sqrt(rng.uniform(0, 1, nb))
    dr, dv = workloads._kepler_relative(rng, mt, a, e)
    r = np.linalg.norm(dr, axis=1)
    v2 = (dv ** 2).sum(axis=1)
    a_rec = 1.0 / (2.0 / r - v2 / mt)
    np.testing.assert_allclose(a_rec, a, rtol=1e-9)
    h = np.cross(dr, dv)
    e_rec = np.sqrt(np.maximum(0.0, 1.0 - (h ** 2).sum(axis=1) / (mt * a)))
    np.testing.assert_allclose(e_rec, e, atol=1e-6)
    assert stats.kstest(e_rec ** 2, "uniform").pvalue > 1e-3  # thermal: e^2 uniform


def test_determinism_and_sizes():
    c1 = workloads.make_cluster(1000, 7, imf=True, binary_fraction=0.2)
    c2 = workloads.make_cluster(1000, 7, imf=True, binary_fraction=0.2)
    assert np.array_equal(c1.pos, c2.pos) and np.array_equal(c1.mass, c2.mass)
    sizes = workloads.batched_sizes(0)
    assert sizes.size == 128 and sizes.min() >= 1024 and sizes.max() <= 131072
    idx = workloads.sample_indices(1000, 100, 0)
    assert np.unique(idx).size == 100


def test_binary_pairs_are_the_generated_binaries():
    """pairs lists each binary's two members once: distinct particles, bound,
    with semi-major axes inside the drawn range."""
    c = workloads.make_cluster(3000, 9, imf=True, binary_fraction=0.5)
    p = c.pairs
    assert p.shape == (c.n_binaries, 2)
    assert len(np.unique(p)) == 2 * c.n_binaries
    r = np.linalg.norm(c.pos[:, p[:, 1]] - c.pos[:, p[:, 0]], axis=0)
    v2 = ((c.vel[:, p[:, 1]] - c.vel[:, p[:, 0]]) ** 2).sum(axis=0)
    mt = c.mass[p[:, 0]] + c.mass[p[:, 1]]
    eps = 0.5 * v2 - mt / r
    assert np.all(eps < 0)
    a = -mt / (2 * eps)
    assert np.all(a > 1e-5 * (1 - 1e-9)) and np.all(a < 1e-2 * (1 + 1e-9))
    assert workloads.make_cluster(100, 1, binary_fraction=0.0).pairs.shape == (0, 2)
