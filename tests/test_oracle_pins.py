"""Pins of the FP64 oracle against what the PeTar paper and the mathematics fix.

None of these tests re-types the oracle's formulas: each checks a property
the paper states (boundary values eq. cof, the relations between f, W and K,
symmetric pair radii), a physical identity (force = -grad potential,
H_L + H_S = Newton, momentum conservation, superposition), a closed form
(two-body branches, quadrupole of two point masses, the (l/d)^3 law of a
quadrupole expansion) or brute force on tiny inputs.
"""

import math
import sys
import os

import numpy as np
import pytest

import workloads

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def _lam(rin, rout):
    return (rout - rin) / (rout + rin)


# ------------------------------------------------------------- changeover

def test_lambda_ratio10_golden():
    g = {k: float(v) for k, v in _read_golden("changeover_ratio10.txt")}
    assert _lam(g["r_in"], g["r_out"]) == pytest.approx(g["lambda_num"] / g["lambda_den"], rel=1e-15)


def _deriv(fn, x, order, h):
    """Central finite difference of the given order (one-sided where needed)."""
    if order == 0:
        return fn(x)
    if order == 1:
        return (fn(x + h) - fn(x - h)) / (2 * h)
    if order == 2:
        return (fn(x + h) - 2 * fn(x) + fn(x - h)) / h ** 2
    if order == 3:
        return (fn(x + 2 * h) - 2 * fn(x + h) + 2 * fn(x - h) - fn(x - 2 * h)) / (2 * h ** 3)
    raise ValueError(order)


@pytest.mark.parametrize("lam", [9 / 11, 0.5, 0.1])
def test_changeover_boundary_values_eq_cof(orc, lam):
    """eq. cof: W(1)=0, K(0)=1, K(1)=0 and K', K'', K''' vanish at 0 and 1.

    Derivatives are taken by finite differences across the boundary, so a
    kink or jump in any of the first three derivatives fails."""
    fns = {"W": lambda x: orc.W(x, lam), "K": lambda x: orc.K(x, lam)}
    for fname, order, x, value in _read_golden("changeover_boundary.txt"):
        order, x, value = int(order), float(x), float(value)
        h = 1e-3
        got = _deriv(fns[fname], x, order, h)
        # K has a 4th-order contact (coefficient <= 35(1+Lambda) < 71), so a
        # difference quotient of order n is off by about 71 (2h)^4 / h^n;
        # a missing or wrong term leaves an O(1..100) derivative instead.
        tol = {0: 1e-15, 1: 1e-6, 2: 1e-3, 3: 0.6}[order]
        assert abs(got - value) <= tol, (fname, order, x, got)


@pytest.mark.parametrize("lam", [9 / 11, 0.3])
def test_changeover_fourth_order_contact(orc, lam):
    """K meets its constant branches with a 4th-order contact (eq. cof):
    (1-K(h))/h^4 and K(1-h)/h^4 converge as h -> 0 (no lower-order term)."""
    for f0 in (lambda h: (1 - orc.K(h, lam)) / h ** 4, lambda h: orc.K(1 - h, lam) / h ** 4):
        vals = [f0(h) for h in (4e-3, 2e-3, 1e-3)]
        d1, d2 = vals[0] - vals[1], vals[1] - vals[2]
        assert np.isfinite(vals).all()
        assert abs(d2) < 0.6 * abs(d1) + 1e-6  # linear convergence in h


@pytest.mark.parametrize("rin,rout", [(1.0, 10.0), (0.002, 0.02), (0.3, 0.5)])
def test_K_from_f_relation(orc, rin, rout):
    """K(x) = f(x) - (x + r_in/(r_out - r_in)) f'(x) for 0 < x < 1 (paper's
    relation between the force weight and f); f' by central differences."""
    lam = _lam(rin, rout)
    c = rin / (rout - rin)
    for x in np.linspace(0.01, 0.99, 99):
        h = 1e-5
        fp = (orc.f(x + h, lam) - orc.f(x - h, lam)) / (2 * h)
        expect = orc.f(x, lam) - (x + c) * fp
        assert orc.K(x, lam) == pytest.approx(expect, abs=1e-9)


@pytest.mark.parametrize("rin,rout", [(1.0, 10.0), (0.002, 0.02)])
def test_W_from_f_relation(orc, rin, rout):
    """W(x) = f(x) - f(1) r/r_out for 0 < x < 1 (offset that makes W(1)=0)."""
    lam = _lam(rin, rout)
    for x in np.linspace(0.0, 1.0, 101)[1:-1]:
        r = rin + x * (rout - rin)
        assert orc.W(x, lam) == pytest.approx(orc.f(x, lam) - orc.f(1.0, lam) * r / rout,
                                               abs=1e-13)


def test_W_K_continuity(orc):
    lam = 9 / 11
    for fn in (orc.W, orc.K):
        for x0 in (0.0, 1.0):
            assert fn(x0 - 1e-12, lam) == pytest.approx(fn(x0 + 1e-12, lam), abs=1e-10)


# ------------------------------------------------------------ two-body pair

def _two_body(orc, r, rin=0.01, rout=0.1, m=0.7, axis=0):
    pos = np.zeros((3, 2))
    pos[axis, 0] = r
    mass = np.array([1.3, m])
    ri = np.array([rin, rin * 0.5])   # pair radii take the max over i, j
    ro = np.array([rout * 0.6, rout])
    return orc.force_long(pos, mass, ri, ro, idx=[0])


def test_two_body_branches(orc):
    """Closed forms per branch of the changeover (x <= 0, x >= 1) and the
    coincident pair (r = 0): no force, finite potential -2Gm/(r_in + r_out)."""
    rin, rout, m = 0.01, 0.1, 0.7
    for r in (0.0, 0.001, 0.005, 0.01):
        a, p = _two_body(orc, r, rin, rout, m)
        assert np.all(a == 0.0)
        assert p[0] == pytest.approx(-2 * m / (rin + rout), rel=1e-14)
    for r in (0.1, 0.2, 3.0):
        a, p = _two_body(orc, r, rin, rout, m)
        assert a[0, 0] == pytest.approx(-m / r ** 2, rel=1e-14)
        assert p[0] == pytest.approx(-m / r, rel=1e-14)


def test_pair_force_is_minus_gradient_of_potential(orc):
    """The long-range pair force is -d(phi_L)/dr throughout the changeover:
    this ties K (force weight) to W (potential weight)."""
    for r in np.linspace(0.0125, 0.0975, 18):
        h = 1e-5  # fourth-order central difference
        ph = [_two_body(orc, r + k * h)[1][0] for k in (-2, -1, 1, 2)]
        a, _ = _two_body(orc, r)
        dphi = (ph[0] - 8 * ph[1] + 8 * ph[2] - ph[3]) / (12 * h)
        assert a[0, 0] == pytest.approx(-dphi, rel=1e-6, abs=1e-9)


def test_pair_radii_symmetric(orc):
    """r_in,ij and r_out,ij take the max over i and j, so the pair force is
    antisymmetric even with unequal radii."""
    pos = np.array([[0.0, 0.03], [0.0, 0.01], [0.0, -0.02]])
    mass = np.array([0.3, 0.9])
    ri = np.array([0.005, 0.02])
    ro = np.array([0.15, 0.05])
    a, _ = orc.force_long(pos, mass, ri, ro)
    np.testing.assert_allclose(mass[0] * a[:, 0], -mass[1] * a[:, 1], rtol=1e-14)


# ----------------------------------------------------------- many-body sums

def _clustered(n, seed):
    c = workloads.make_cluster(n, seed, imf=True, binary_fraction=0.5, a_min=1e-3, a_max=3e-2)
    return c


def test_long_plus_short_is_newton(orc):
    """H = H_L + H_S (eq. cf): a_L + a_S = a_Newton and phi_L + phi_S = phi_N,
    from three independent loops."""
    c = _clustered(300, 3)
    rin, rout, rs = orc.radii(c.mass, 0.01, 0.1)
    aL, pL = orc.force_long(c.pos, c.mass, rin, rout)
    aS, pS = orc.force_short(c.pos, c.mass, rin, rout)
    aN, pN = orc.force_newton(c.pos, c.mass)
    scale = np.linalg.norm(aN, axis=0)
    err = np.linalg.norm(aL + aS - aN, axis=0) / scale
    assert err.max() < 1e-12
    np.testing.assert_allclose(pL + pS, pN, rtol=1e-12)
    # the split is non-trivial for this input
    assert np.linalg.norm(aS, axis=0).max() > 1e-3 * scale.max()


def test_momentum_conservation(orc):
    """Pair forces are antisymmetric, so sum_i m_i a_L,i = 0."""
    c = _clustered(400, 4)
    rin, rout, _ = orc.radii(c.mass, 0.005, 0.05)
    a, _ = orc.force_long(c.pos, c.mass, rin, rout)
    tot = (c.mass[None, :] * a).sum(axis=1)
    assert np.abs(tot).max() < 1e-13 * np.abs(c.mass[None, :] * a).sum()


def test_potential_superposition(orc):
    """1/2 sum_i m_i phi_i equals the sum over pairs i<j of the two-body
    potential energy (self pairs excluded)."""
    c = _clustered(24, 5)
    rin, rout, _ = orc.radii(c.mass, 0.02, 0.2)
    _, phi = orc.force_long(c.pos, c.mass, rin, rout)
    e_pairs = 0.0
    n = c.mass.size
    for i in range(n):
        for j in range(i + 1, n):
            sel = [i, j]
            _, p2 = orc.force_long(c.pos[:, sel], c.mass[sel], rin[sel], rout[sel], idx=[0])
            e_pairs += c.mass[i] * p2[0]
    assert 0.5 * np.dot(c.mass, phi) == pytest.approx(e_pairs, rel=1e-13)


def test_coincident_particles(orc):
    """r = 0 pairs: a_L = 0 from that pair and phi stays finite."""
    pos = np.array([[0.1, 0.1, 0.5], [0.2, 0.2, 0.0], [0.3, 0.3, 0.0]])
    mass = np.array([0.2, 0.3, 0.5])
    rin, rout = np.full(3, 0.01), np.full(3, 0.1)
    a, p = orc.force_long(pos, mass, rin, rout)
    assert np.isfinite(a).all() and np.isfinite(p).all()
    # particle 0 only feels particle 2 (Newtonian: distance 0.5 > r_out)
    d = pos[:, 2] - pos[:, 0]
    np.testing.assert_allclose(a[:, 0], mass[2] * d / np.linalg.norm(d) ** 3, rtol=1e-14)
    assert p[0] == pytest.approx(-mass[1] * 2 / 0.11 - mass[2] / np.linalg.norm(d), rel=1e-14)


# --------------------------------------------------------------------- radii

def test_radii_eq_rcut(orc):
    """eq. rcut: factor max(1, m/<m>)^(1/3); eq. rnb for the search radius."""
    mass = np.array([1.0, 1.0, 8.0, 27.0, 0.5, 0.5, 0.5, 0.5])
    mave = mass.mean()
    rin, rout, rs = orc.radii(mass, 0.01, 0.1, search_factor=1.2)
    s = np.array([max(1.0, m / mave) ** (1 / 3) for m in mass])
    np.testing.assert_allclose(rin, 0.01 * s, rtol=1e-15)
    np.testing.assert_allclose(rout, 0.1 * s, rtol=1e-15)
    np.testing.assert_allclose(rs, 0.12 * s, rtol=1e-15)
    # equal masses: factor exactly 1
    rin, rout, rs = orc.radii(np.full(16, 1 / 16), 0.01, 0.1, 1.2)
    assert np.all(rin == 0.01) and np.all(rout == 0.1)
    # eq. rnb: r_nb = r_out + C_r |v| dt
    vel = np.zeros((3, 8))
    vel[0] = np.arange(8)
    rin, rout, rs = orc.radii(mass, 0.01, 0.1, vel=vel, cr_dt=3.0 / 1024)
    np.testing.assert_allclose(rs, rout + 3.0 / 1024 * np.arange(8), rtol=1e-15)


# ---------------------------------------------------------------- neighbours

def _brute_nb(pos, rs):
    n = rs.size
    out = []
    for i in range(n):
        lst = []
        for j in range(n):
            if j == i:
                continue
            d = [pos[k, j] - pos[k, i] for k in range(3)]
            d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
            R = max(rs[i], rs[j])
            if d2 < R * R:
                lst.append(j)
        out.append(lst)
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_neighbours_brute_force(orc, seed):
    rng = np.random.default_rng(seed)
    n = 48
    pos = rng.uniform(-0.2, 0.2, (3, n))
    rs = rng.uniform(0.02, 0.15, n)
    # adversarial: pairs at exactly R on an axis, and a duplicate position
    pos[:, 1] = pos[:, 0]
    pos[:, 3] = pos[:, 2]
    pos[0, 3] += max(rs[2], rs[3])
    offs, idx = orc.neighbours(pos, rs)
    ref = _brute_nb(pos, rs)
    for i in range(n):
        assert list(idx[offs[i]:offs[i + 1]]) == ref[i]
    assert 1 in list(idx[offs[0]:offs[1]])          # duplicate is a neighbour
    # permutation invariance of the neighbour relation
    perm = rng.permutation(n)
    offs2, idx2 = orc.neighbours(pos[:, perm], rs[perm])
    inv = np.argsort(perm)
    for i in range(n):
        got = sorted(perm[idx2[offs2[inv[i]]:offs2[inv[i] + 1]]])
        assert got == ref[i]


def test_neighbours_symmetric(orc):
    c = _clustered(500, 9)
    _, _, rs = orc.radii(c.mass, 0.01, 0.1)
    offs, idx = orc.neighbours(c.pos, rs)
    pairs = set()
    for i in range(500):
        for j in idx[offs[i]:offs[i + 1]]:
            pairs.add((i, int(j)))
    assert all((j, i) in pairs for (i, j) in pairs)
    assert len(pairs) > 0


# ---------------------------------------------------------------- multipoles

def test_quadrupole_two_point_masses(orc):
    """Two masses m at +-d z: A' = diag(-m d^2, -m d^2, 2 m d^2) (eq. quadtr)."""
    m, d = 0.25, 0.3
    pos = np.array([[0.0, 0.0], [0.0, 0.0], [d, -d]])
    M, com, q = orc.multipole(pos, np.array([m, m]))
    assert M == 0.5 and np.allclose(com, 0)
    np.testing.assert_allclose(q, [-m * d * d, -m * d * d, 2 * m * d * d, 0, 0, 0], atol=1e-16)


def test_quadrupole_error_law(orc):
    """With the centre of mass as expansion point and the quadrupole kept,
    the field error of a compact cluster falls as (l/d)^3 relative; a missing
    or wrong quadrupole leaves an (l/d)^2 error."""
    rng = np.random.default_rng(11)
    n = 64
    pos = rng.uniform(-0.5, 0.5, (3, n)) * np.array([[1.0], [0.6], [0.3]])
    mass = rng.uniform(0.5, 1.5, n)
    M, com, q = orc.multipole(pos, mass)
    dirs = workloads._isotropic(rng, 20).T
    errs = []
    for dist in (8.0, 16.0, 32.0):
        pts = com[:, None] + dist * dirs
        a_ex = np.empty((3, 20))
        for k in range(20):
            allp = np.concatenate([pts[:, k:k + 1], pos], axis=1)
            allm = np.concatenate([[0.0], mass])
            a, _ = orc.force_newton(allp, allm, idx=[0])
            a_ex[:, k] = a[:, 0]
        a_mp, _ = orc.multipole_eval(M, com, q, pts)
        errs.append(np.median(np.linalg.norm(a_mp - a_ex, axis=0) / np.linalg.norm(a_ex, axis=0)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 6.0 < r1 < 10.5 and 6.0 < r2 < 10.5, errs


# ---------------------------------------------------------------------- tree

def test_tree_theta0_is_direct_sum(orc):
    """theta = 0 opens every cell, so the tree reaches exactly the direct
    sum's pair set."""
    c = workloads.make_cluster(3000, 21, imf=True, binary_fraction=0.5)
    rin, rout, rs = orc.radii(c.mass, 0.005, 0.05)
    a0, p0 = orc.force_long(c.pos, c.mass, rin, rout)
    for leaf, grp in ((8, 64), (1, 1), (16, 200)):
        at, pt, cnt = orc.tree_force(c.pos, c.mass, rin, rout, rs, 0.0, leaf, grp)
        err = np.linalg.norm(at - a0, axis=0) / np.linalg.norm(a0, axis=0)
        assert err.max() < 1e-11
        np.testing.assert_allclose(pt, p0, rtol=1e-12)
        assert np.all(cnt[0] == 0)
        assert np.all(cnt[1] + cnt[2] == 3000)


def _with_massless(orc, n, seed):
    """A cluster where some particles have no mass: a clump of 300 massless
    particles off to one side (whole cells of zero mass) and a third of the
    others scattered through the cluster."""
    c = workloads.make_cluster(n, seed, imf=True, binary_fraction=0.5)
    rng = np.random.default_rng(seed)
    pos, mass = c.pos.copy(), c.mass.copy()
    pos[:, :300] = rng.normal(scale=0.02, size=(3, 300)) + np.array([[1.5], [0.0], [0.0]])
    mass[:300] = 0.0
    mass[300:][rng.random(n - 300) < 1.0 / 3.0] = 0.0
    rin, rout, rs = orc.radii(np.maximum(mass, 1e-6), 0.005, 0.05)
    return pos, mass, rin, rout, rs


def test_tree_skip_massless_changes_no_value(orc):
    """Dropping the cells of zero mass from the walk and the particles of
    zero mass from the leaf lists (the rule of a force on a subset of
    targets) leaves every acceleration and potential bit for bit as it was,
    at theta 0 still equal to the direct sum, and only lowers the
    interaction counts: at theta 0 each target's particle lists hold exactly
    the particles with mass."""
    pos, mass, rin, rout, rs = _with_massless(orc, 3000, 25)
    idx = np.arange(0, 3000, 3)
    for theta in (0.0, 0.5):
        a1, p1, c1 = orc.tree_force(pos, mass, rin, rout, rs, theta, 8, 64, idx=idx)
        a2, p2, c2 = orc.tree_force(pos, mass, rin, rout, rs, theta, 8, 64, idx=idx,
                                    skip_massless=True)
        assert np.array_equal(a1, a2) and np.array_equal(p1, p2)
        assert np.all(c2[:3] <= c1[:3]) and c2[:3].sum() < c1[:3].sum()
        assert np.array_equal(c2[3], c1[3])
    a0, p0 = orc.force_long(pos, mass, rin, rout, idx=idx)
    err = np.linalg.norm(a2 - a0, axis=0) / np.linalg.norm(a0, axis=0)
    a0t, _, c0t = orc.tree_force(pos, mass, rin, rout, rs, 0.0, 8, 64, idx=idx,
                                 skip_massless=True)
    # at theta 0 every leaf is reached: the far and near lists of each target
    # hold every particle with mass once (and every particle without the rule)
    _, _, c0 = orc.tree_force(pos, mass, rin, rout, rs, 0.0, 8, 64, idx=idx)
    assert np.all(c0t[0] == 0) and np.all(c0t[1] + c0t[2] == np.count_nonzero(mass))
    assert np.all(c0[1] + c0[2] == mass.size)
    # with every mass nonzero the rule changes nothing, the counts included
    m1 = np.where(mass == 0.0, 1e-7, mass)
    r1 = orc.tree_force(pos, m1, rin, rout, rs, 0.5, 8, 64, idx=idx)
    r2 = orc.tree_force(pos, m1, rin, rout, rs, 0.5, 8, 64, idx=idx, skip_massless=True)
    assert all(np.array_equal(x, y) for x, y in zip(r1, r2))
    err0 = np.linalg.norm(a0t - a0, axis=0) / np.linalg.norm(a0, axis=0)
    assert err0.max() < 1e-11 and err.max() < 1e-2


def test_tree_error_decreases_with_theta(orc):
    c = workloads.make_cluster(4096, 0, imf=False)
    rin, rout, rs = np.full(4096, 0.01), np.full(4096, 0.1), np.full(4096, 0.12)
    a0, _ = orc.force_long(c.pos, c.mass, rin, rout)
    med = []
    for th in (0.2, 0.4, 0.7):
        at, _, _ = orc.tree_force(c.pos, c.mass, rin, rout, rs, th, 8, 64)
        med.append(np.median(np.linalg.norm(at - a0, axis=0) / np.linalg.norm(a0, axis=0)))
    assert med[0] < med[1] < med[2] < 3e-3


def test_tree_structure_and_max_depth(orc):
    """Each particle in exactly one leaf; more than leaf_size coincident
    particles end in one leaf at the deepest level."""
    c = workloads.make_cluster(1000, 5, imf=True)
    info = orc.tree_info(c.pos, c.mass, 8, 64)
    assert info["sum_leaf"] == 1000 and info["max_leaf"] <= 8
    pos = c.pos.copy()
    pos[:, :20] = pos[:, :1]
    info = orc.tree_info(pos, c.mass, 8, 64)
    assert info["sum_leaf"] == 1000 and info["max_level"] == 21 and info["max_leaf"] == 20


def test_tree_near_list_holds_neighbours(orc):
    """Walk conservativeness: every pair within r_search is a near pair, so
    with theta = 0.7 the tree force still matches the direct sum on the
    changeover part (checked through the short-range split)."""
    c = workloads.make_cluster(2000, 8, imf=True, binary_fraction=1.0, a_min=1e-3, a_max=2e-2)
    rin, rout, rs = orc.radii(c.mass, 0.005, 0.05)
    at, pt, cnt = orc.tree_force(c.pos, c.mass, rin, rout, rs, 0.7, 8, 32)
    offs, _ = orc.neighbours(c.pos, rs)
    # near particles per target (including itself) cover its neighbours
    assert np.all(cnt[2] >= np.diff(offs) + 1)


# ------------------------------------------- second stage and clusters
def _rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    return q * np.sign(np.diag(r))


def _conic_state(p, e, f, mu, rng):
    """Relative state of a Kepler conic with semi-latus rectum p and
    eccentricity e at true anomaly f (polar form r = p/(1 + e cos f), radial
    and transverse speeds sqrt(mu/p) e sin f and sqrt(mu/p)(1 + e cos f)),
    rotated and translated at random."""
    r = p / (1.0 + e * math.cos(f))
    s = math.sqrt(mu / p)
    vr, vt = s * e * math.sin(f), s * (1.0 + e * math.cos(f))
    rhat = np.array([math.cos(f), math.sin(f), 0.0])
    that = np.array([-math.sin(f), math.cos(f), 0.0])
    Q = _rotation(rng)
    x = Q @ (r * rhat)
    v = Q @ (vr * rhat + vt * that)
    x0, v0 = rng.normal(size=3), rng.normal(size=3)
    return x0, v0, x0 + x, v0 + v


@pytest.mark.parametrize("e", [0.0, 0.3, 0.9, 0.999, 1.0, 1.7, 12.0])
def test_pericentre_of_conics(orc, e):
    """r_p = p / (1 + e) for ellipses, the parabola and hyperbolae, at any
    phase of the orbit (the pericentre of the whole orbit)."""
    rng = np.random.default_rng(int(e * 1000) + 1)
    for f in (0.0, 0.7, 2.0, -1.3):
        if e >= 1.0 and 1.0 + e * math.cos(f) <= 0.05:
            continue  # outside the branch of an open orbit
        mu, p = 0.8, 0.37
        xi, vi, xj, vj = _conic_state(p, e, f, mu, rng)
        mi = 0.3
        rp = orc.pericentre(xi, vi, mi, xj, vj, mu - mi, 1.0)
        # near e = 0 the eccentricity is the root of a rounding-level number
        tol = 1e-9 if e >= 0.3 else 3e-8
        assert abs(rp / (p / (1.0 + e)) - 1.0) < tol, (e, f, rp)


def test_pericentre_special_cases(orc):
    x0, v0 = np.array([0.1, -0.2, 0.3]), np.array([0.5, 0.1, -0.2])
    # radial motion: zero angular momentum
    assert orc.pericentre(x0, v0, 0.5, x0 + [1.0, 0, 0], v0 + [0.3, 0, 0], 0.5) == 0.0
    # coincident particles
    assert orc.pericentre(x0, v0, 0.5, x0, v0 + [1.0, 2.0, 0], 0.5) == 0.0
    # massless pair: straight lines, closest approach = impact parameter
    rp = orc.pericentre(x0, v0, 0.0, x0 + [2.0, 0.25, 0], v0 + [-1.0, 0, 0], 0.0)
    assert abs(rp - 0.25) < 1e-15
    rp = orc.pericentre(x0, v0, 0.0, x0 + [0.0, 0.4, 0.3], v0, 0.0)
    assert abs(rp - 0.5) < 1e-15
    # circular orbit: r_p = r
    rp = orc.pericentre([0, 0, 0], [0, 0, 0], 0.25, [2.0, 0, 0], [0, math.sqrt(0.5 / 2.0), 0],
                        0.25)
    assert abs(rp - 2.0) < 1e-14
    # symmetric in the pair, bit for bit
    rng = np.random.default_rng(3)
    for _ in range(50):
        a, b, c, d = rng.normal(size=(4, 3))
        assert orc.pericentre(a, b, 0.3, c, d, 0.6) == orc.pericentre(c, d, 0.6, a, b, 0.3)


def test_nb_filter_selects_by_pericentre(orc):
    """Second stage on a real candidate list: j is kept in i's list iff its
    pericentre is below c_v * r_nb,i; list order is kept."""
    c = workloads.make_cluster(3000, 31, imf=True, binary_fraction=0.5)
    rin, rout, rnb = orc.radii(c.mass, 0.005, 0.05, vel=c.vel, cr_dt=3.0 * 0.003)
    offs, idx = orc.neighbours(c.pos, rnb)
    f_offs, f_idx = orc.nb_filter(c.pos, c.vel, c.mass, rnb, 1.5, offs, idx)
    p, v = c.pos.T, c.vel.T
    kept = dropped = 0
    for i in range(3000):
        want = [j for j in idx[offs[i]:offs[i + 1]]
                if orc.pericentre(p[i], v[i], c.mass[i], p[j], v[j], c.mass[j]) < 1.5 * rnb[i]]
        got = list(f_idx[f_offs[i]:f_offs[i + 1]])
        assert got == want
        kept += len(want)
        dropped += offs[i + 1] - offs[i] - len(want)
    assert kept > 0 and dropped > 0


def _components_bfs(n, offs, idx):
    adj = [set() for _ in range(n)]
    for i in range(n):
        for j in idx[offs[i]:offs[i + 1]]:
            adj[i].add(int(j))
            adj[int(j)].add(i)
    label = [-1] * n
    for s in range(n):
        if label[s] >= 0:
            continue
        stack, comp = [s], []
        label[s] = s
        while stack:
            u = stack.pop()
            comp.append(u)
            for w in adj[u]:
                if label[w] < 0:
                    label[w] = s
                    stack.append(w)
    return np.array(label, dtype=np.int32)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_clusters_are_connected_components(orc, seed):
    """Labels equal breadth-first components (label = smallest member);
    directed lists are closed under the cluster; the cluster CSR lists each
    cluster by label with members ascending."""
    rng = np.random.default_rng(seed)
    n = 400
    lists = []
    for i in range(n):
        k = int(rng.integers(0, 3)) if rng.random() < 0.6 else 0
        lists.append(sorted(set(int(j) for j in rng.integers(0, n, size=k) if j != i)))
    offs = np.zeros(n + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(l) for l in lists])
    idx = np.array([j for l in lists for j in l], dtype=np.int32)
    label, cl, members = orc.clusters(n, offs, idx)
    assert np.array_equal(label, _components_bfs(n, offs, idx))
    for i in range(n):
        assert all(label[j] == label[i] for j in idx[offs[i]:offs[i + 1]])
    roots = np.unique(label)
    assert cl.size == roots.size + 1 and cl[-1] == n
    for k, r in enumerate(roots):
        mem = members[cl[k]:cl[k + 1]]
        assert mem[0] == r and np.all(np.diff(mem) > 0) and np.all(label[mem] == r)


# ------------------------------------------------- artificial particles
_TT_NAMES = ["xx", "xy", "xz", "yy", "yz", "zz", "xxx", "xxy", "xxz", "xyy", "xyz", "xzz",
             "yyy", "yyz", "yzz", "zzz"]


def test_tidal_generalized_inverse_equals_table_a(orc):
    """The least-squares inverse of the measure-point map reproduces the
    printed closed forms of Table A, row by row."""
    def value(text):
        # the paper's printed form: +-a/b or +-sqrt2/b
        sign = -1.0 if text[0] == "-" else 1.0
        num, den = text.lstrip("+-").split("/")
        top = math.sqrt(2.0) if num == "sqrt2" else float(num)
        return sign * top / float(den)

    rows = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "tidal_table_a.txt")):
        if line.startswith("#") or not line.strip():
            continue
        order, name, point, comp, val = line.split()
        rows.setdefault((int(order), name), {})[(int(point) - 1, "xyz".index(comp))] = value(val)
    # every row of both blocks of the table
    assert sorted(k for k in rows if k[0] == 2) == sorted((2, nm) for nm in _TT_NAMES[:6])
    assert sorted(k for k in rows if k[0] == 3) == sorted((3, nm) for nm in _TT_NAMES)
    for (order, name), want in rows.items():
        g = orc.tidal_ginv(order)[_TT_NAMES.index(name)]
        got = {(r // 3, r % 3): v for r, v in enumerate(g) if abs(v) > 1e-14}
        assert set(got) == set(want), (order, name)
        for key, v in want.items():
            assert abs(got[key] - v) < 1e-15, (order, name, key)


def test_tidal_condition_numbers(orc):
    """Condition numbers of the normal matrices of the maps: 2 and 12.7
    (the values the paper quotes)."""
    for order, want, tol in ((2, 2.0, 1e-12), (3, 12.7, 0.05)):
        M = np.linalg.pinv(orc.tidal_ginv(order))
        s = np.linalg.svd(M.T @ M, compute_uv=False)
        assert abs(s.max() / s.min() - want) < tol, (order, s.max() / s.min())


@pytest.mark.parametrize("order", [2, 3])
def test_tidal_fit_recovers_polynomial_fields(orc, order):
    """A field that is exactly of the model's form is recovered exactly
    (up to rounding), at any d_c; the points sit at d_c times Table A's
    offsets around the centre."""
    rng = np.random.default_rng(order)
    K = 6 if order == 2 else 16
    t = rng.normal(size=3 + K)
    cm, d_c = rng.normal(size=3), 0.0123
    pts = orc.tidal_points(order, cm, d_c)
    u = (pts - cm) / d_c
    s2 = math.sqrt(2.0) / 2.0
    ref_u = (np.array([[1, 0, -s2], [-1, 0, -s2], [0, 1, s2], [0, -1, s2]]) if order == 2 else
             np.array([[1, 0, -1], [0, 1, -1], [-1, 0, -1], [0, -1, -1], [1, 0, 1], [0, 1, 1],
                       [-1, 0, 1], [0, -1, 1]]))
    assert np.allclose(u, ref_u, atol=1e-12)
    acc = np.array([orc.tidal_eval(order, t, p - cm) for p in pts])
    fit = orc.tidal_fit(order, d_c, t[:3], acc)
    assert np.allclose(fit, t, rtol=1e-8, atol=1e-9)


def test_tidal_fit_of_point_mass_field(orc):
    """Measure points near r = 0 in the field of a distant unit mass: the
    fitted gradient is the Newtonian tidal tensor G m (3 n n^T - I)/D^3 up
    to the truncation of the model (relative d_c / D for order 2,
    (d_c / D)^2 for order 3)."""
    D = np.array([3.0, -1.0, 2.0])
    dn = np.linalg.norm(D)
    n = D / dn

    def field(p):
        r = D - p
        return r / np.linalg.norm(r) ** 3

    tid = (3.0 * np.outer(n, n) - np.eye(3)) / dn ** 3
    want = np.array([tid[0, 0], tid[0, 1], tid[0, 2], tid[1, 1], tid[1, 2], tid[2, 2]])
    for order, d_c in ((2, 1e-3), (3, 1e-2)):
        cm = np.zeros(3)
        pts = orc.tidal_points(order, cm, d_c)
        fit = orc.tidal_fit(order, d_c, field(cm), np.array([field(p) for p in pts]))
        err = np.abs(fit[3:9] - want).max() / np.abs(want).max()
        bound = 10 * (d_c / dn) ** (order - 1)
        assert err < bound, (order, err, bound)


def _binary_from_elements(a, e, m1, m2, Q, E0, G=1.0):
    M = m1 + m2
    n = math.sqrt(G * M / a ** 3)
    r_orb = np.array([a * (math.cos(E0) - e), a * math.sqrt(1 - e * e) * math.sin(E0), 0.0])
    fac = n / (1.0 - e * math.cos(E0))
    v_orb = np.array([-a * math.sin(E0) * fac, a * math.sqrt(1 - e * e) * math.cos(E0) * fac, 0.0])
    r, v = Q @ r_orb, Q @ v_orb
    cm, vcm = np.array([0.3, -0.2, 0.1]), np.array([0.05, 0.0, -0.1])
    return (cm - m2 / M * r, cm + m1 / M * r, vcm - m2 / M * v, vcm + m1 / M * v, cm)


@pytest.mark.parametrize("e", [0.0, 0.3, 0.8, 0.97])
def test_pseudo_particles_carry_orbit_averaged_quadrupole(orc, e):
    """The three pseudoparticles have the binary's mass and centre of mass,
    and their second moment about it equals the time average of the
    binary's second moment over one orbit, computed by quadrature in the
    eccentric anomaly (dt proportional to 1 - e cos E)."""
    rng = np.random.default_rng(int(e * 100))
    m1, m2, a = 0.7, 0.4, 0.013
    Q = _rotation(rng)
    x1, x2, v1, v2, cm = _binary_from_elements(a, e, m1, m2, Q, 1.1)
    pos, mp = orc.pseudo_particles(m1, m2, x1, x2, v1, v2)
    assert abs(3 * mp - (m1 + m2)) < 1e-15
    assert np.allclose(pos.mean(axis=0), cm, atol=1e-14)
    got = mp * sum(np.outer(p - cm, p - cm) for p in pos)
    Es = np.linspace(0, 2 * math.pi, 4001)[:-1]
    w = (1 - e * np.cos(Es))
    acc = np.zeros((3, 3))
    for E, wi in zip(Es, w):
        r = Q @ np.array([a * (math.cos(E) - e), a * math.sqrt(1 - e * e) * math.sin(E), 0.0])
        r1, r2 = -m2 / (m1 + m2) * r, m1 / (m1 + m2) * r
        acc += wi * (m1 * np.outer(r1, r1) + m2 * np.outer(r2, r2))
    want = acc / w.sum()
    assert np.allclose(got, want, rtol=0, atol=1e-10 * np.abs(want).max())


def test_pseudo_particles_reject_unbound(orc):
    x1, x2 = np.zeros(3), np.array([1.0, 0, 0])
    assert orc.pseudo_particles(0.5, 0.5, x1, x2, np.zeros(3), np.array([0, 2.0, 0])) is None
    assert orc.pseudo_particles(0.5, 0.5, x1, x2, np.zeros(3), np.array([0, 0.5, 0])) is not None


def test_pseudo_particles_traceless_closed_form(orc):
    """The traceless form of the pseudoparticles' second moment equals the
    closed form mu a^2 / 4 diag(9e^2 + 1, 1 - 6e^2, -3e^2 - 2) in the frame
    (x to the pericentre, z along the angular momentum)."""
    m1, m2, a, e = 0.3, 0.9, 0.02, 0.6
    Q = np.eye(3)
    x1, x2, v1, v2, cm = _binary_from_elements(a, e, m1, m2, Q, 2.3)
    pos, mp = orc.pseudo_particles(m1, m2, x1, x2, v1, v2)
    A = mp * sum(np.outer(p - cm, p - cm) for p in pos)
    At = 1.5 * A - 0.5 * np.trace(A) * np.eye(3)
    mu = m1 * m2 / (m1 + m2)
    want = mu * a * a / 4 * np.diag([9 * e * e + 1, 1 - 6 * e * e, -3 * e * e - 2])
    assert np.allclose(At, want, rtol=0, atol=1e-13 * np.abs(want).max())


def test_pseudo_particles_radial_orbit(orc):
    """Zero angular momentum: the e -> 1 limit, all three points on the
    separation line, second moment mu a^2 (5/2) along it."""
    m1, m2 = 0.4, 0.6
    x1, x2 = np.array([0.0, 0.0, 0.0]), np.array([0.3, 0.4, 0.0])
    v1, v2 = np.zeros(3), np.array([0.6, 0.8, 0.0]) * 0.5
    pos, mp = orc.pseudo_particles(m1, m2, x1, x2, v1, v2)
    a, e = orc.binary_elements(m1, m2, x1, x2, v1, v2)
    assert abs(e - 1.0) < 1e-7
    cm = (m1 * x1 + m2 * x2) / (m1 + m2)
    n = (x2 - x1) / np.linalg.norm(x2 - x1)
    A = mp * sum(np.outer(p - cm, p - cm) for p in pos)
    mu = m1 * m2 / (m1 + m2)
    assert np.allclose(A, 2.5 * mu * a * a * np.outer(n, n), atol=1e-14)


@pytest.mark.parametrize("e", [0.0, 0.5, 0.95])
def test_binary_elements_recovered(orc, e):
    rng = np.random.default_rng(7)
    for E0 in (0.0, 1.0, 3.0):
        x1, x2, v1, v2, _ = _binary_from_elements(0.01, e, 0.2, 0.5, _rotation(rng), E0)
        a, ee = orc.binary_elements(0.2, 0.5, x1, x2, v1, v2)
        assert abs(a - 0.01) < 1e-14 and abs(ee - e) < 1e-7


@pytest.mark.parametrize("order", [2, 3])
def test_tidal_potential_gradient_is_field(orc, order):
    """Minus the gradient of the model potential is the model field (central
    differences; the potential is a polynomial of degree order)."""
    rng = np.random.default_rng(11 + order)
    t = rng.normal(size=3 + (6 if order == 2 else 16))
    r0, h = rng.normal(size=3) * 0.3, 1e-4
    g = np.array([(orc.tidal_potential(order, t, r0 + h * ek, 0.7) -
                   orc.tidal_potential(order, t, r0 - h * ek, 0.7)) / (2 * h) for ek in np.eye(3)])
    assert np.allclose(-g, orc.tidal_eval(order, t, r0), rtol=1e-7, atol=1e-7)
    assert orc.tidal_potential(order, t, np.zeros(3), 0.7) == 0.7


def test_artificial_set_bookkeeping(orc):
    """Members leave the set, singles keep their order and values, every
    pair adds its centre, P measure points and three pseudoparticles; mass
    and the pair's centre of mass are conserved."""
    rng = np.random.default_rng(5)
    n = 12
    pos, vel = rng.normal(size=(3, n)), rng.normal(size=(3, n)) * 0.01
    mass = rng.uniform(0.5, 1.0, n)
    pairs = np.array([[3, 7], [10, 0]])
    for b, (i, j) in enumerate(pairs):
        x1, x2, v1, v2, _ = _binary_from_elements(0.01 * (b + 1), 0.4, mass[i], mass[j],
                                                  _rotation(rng), 0.5 + b)
        pos[:, i], pos[:, j], vel[:, i], vel[:, j] = x1 + b, x2 + b, v1, v2
    r_in, r_out = rng.uniform(0.1, 0.2, n), rng.uniform(0.3, 0.4, n)
    r_s = r_out * 1.2
    for order, P in ((2, 4), (3, 8)):
        art = orc.artificial_set(pos, vel, mass, r_in, r_out, r_s, pairs, order, 0.8)
        singles = [k for k in range(n) if k not in pairs.ravel()]
        assert art["n_single"] == len(singles) and list(art["src"][:len(singles)]) == singles
        assert np.array_equal(art["pos"][:, :len(singles)], pos[:, singles])
        assert art["pos"].shape[1] == len(singles) + 2 * (P + 4)
        assert abs(art["mass"].sum() - mass.sum()) < 1e-14
        for b, (i, j) in enumerate(pairs):
            base = len(singles) + b * (P + 4)
            blk = slice(base, base + P + 4)
            cm = (mass[i] * pos[:, i] + mass[j] * pos[:, j]) / (mass[i] + mass[j])
            m = art["mass"][blk]
            assert np.all(m[:P + 1] == 0) and np.allclose(m[P + 1:], (mass[i] + mass[j]) / 3)
            assert np.allclose(art["pos"][:, blk] @ m / m.sum(), cm, atol=1e-14)
            a, e = orc.binary_elements(mass[i], mass[j], pos[:, i], pos[:, j], vel[:, i],
                                       vel[:, j])
            assert abs(art["frame"][b, 3] - 0.8 * a * (1 + e)) < 1e-15
            d = np.linalg.norm(art["pos"][:, base + 1:base + 1 + P] - cm[:, None], axis=0)
            want = art["frame"][b, 3] * (math.sqrt(1.5) if order == 2 else math.sqrt(2.0))
            assert np.allclose(d, want, rtol=1e-13)
            assert np.all(art["r_in"][blk] == max(r_in[i], r_in[j]))
            assert art["pair_of"][i] == b and art["pair_of"][j] == b
    with pytest.raises(ValueError):
        orc.artificial_set(pos, vel, mass, r_in, r_out, r_s, [[1, 2], [2, 4]], 2, 1.0)


@pytest.mark.parametrize("order", [2, 3])
def test_artificial_pipeline_binary_and_perturber(orc, order):
    """A bound binary deep inside its inner changeover radius and a distant
    perturber outside every outer radius: through the long-range direct sum
    over the artificial set and the post-fit, (1) each member feels the
    perturber's Newtonian field at its own position up to the truncation of
    the tidal model, and (2) the perturber feels the binary's monopole plus
    its orbit-averaged quadrupole (eq. avebinquad) up to the octupole."""
    m1, m2, mp, a, e = 0.6, 0.3, 1.0, 1e-3, 0.5
    rng = np.random.default_rng(order)
    x1, x2, v1, v2, cm = _binary_from_elements(a, e, m1, m2, _rotation(rng), 0.9)
    D = np.array([0.25, -0.1, 0.15])
    pos = np.stack([x1, x2, cm + D], axis=1)
    vel = np.stack([v1, v2, np.zeros(3)], axis=1)
    mass = np.array([m1, m2, mp])
    r_in, r_out = np.full(3, 0.02), np.full(3, 0.1)
    art = orc.artificial_set(pos, vel, mass, r_in, r_out, 1.2 * r_out, [[0, 1]], order, 1.0)
    acc_set, pot_set = orc.force_long(art["pos"], art["mass"], art["r_in"], art["r_out"])
    rec, acc, pot = orc.artificial_fit(order, art, pos, acc_set, pot_set, [[0, 1]])
    dn = np.linalg.norm(D)
    # the pair's own pseudoparticles lie inside r_in of its members: their
    # long-range force vanishes there and their potential is a constant
    P = 4 if order == 2 else 8
    own = art["n_single"] + 1 + P
    sub = np.concatenate([art["pos"][:, own:own + 3], cm[:, None]], axis=1)
    _, pot_own = orc.force_long(sub, np.append(art["mass"][own:own + 3], 0.0), np.full(4, 0.02),
                                np.full(4, 0.1))
    for k in (0, 1):
        r = pos[:, 2] - pos[:, k]
        want = mp * r / np.linalg.norm(r) ** 3
        err = np.linalg.norm(acc[:, k] - want) / np.linalg.norm(want)
        # the model's first dropped term, relative: (|r'| / D)^order; the
        # fit through points at d_c adds the same order
        assert err < 2 * (1.5 * a / dn) ** order, (k, err)
        assert abs(pot[k] + mp / np.linalg.norm(r) - pot_own[3]) < 2 * (1.5 * a / dn) ** order * mp / dn
    M, com, q = orc.multipole(art["pos"][:, art["n_single"]:], art["mass"][art["n_single"]:])
    assert np.allclose(com, cm, atol=1e-15)
    quad_acc, _ = orc.multipole_eval(M, com, q, pos[:, 2:3])
    s = a * math.sqrt(m1 * m2) / (m1 + m2)
    err = np.linalg.norm(acc[:, 2] - quad_acc[:, 0]) / np.linalg.norm(quad_acc[:, 0])
    assert err < (2 * s / dn) ** 3
    # the orbit-averaged quadrupole: the pseudoparticles' second moment
    bin_q = (m1 + m2) / 3 * sum(np.outer(p - cm, p - cm)
                                for p in art["pos"][:, art["n_single"] + 1 + (4 if order == 2 else 8):].T)
    A = bin_q
    mu = m1 * m2 / (m1 + m2)
    assert abs(np.trace(A) - mu * a * a * (1.5 * e * e + 1.0)) < 1e-15


# ------------------------------------------------------------- SDAR groups
def test_groups_constructed_cases(orc):
    """eq. rbin with r_in,ij = max(r_in,i, r_in,j): a chain a-b-c with a-c
    too far is one group of three (the relation is closed transitively), an
    isolated bound pair is a binary, a close but unbound pair is a group but
    no binary, and a pair closer than theta r_in of only the larger-radius
    member still counts."""
    theta = 0.5
    pos = np.array([[0.0, 0.009, 0.018, 5.0, 5.004, 9.0, 9.004, 12.0, 12.009],
                    [0.0] * 9, [0.0] * 9])
    r_in = np.array([0.02, 0.02, 0.02, 0.01, 0.01, 0.01, 0.01, 0.001, 0.02])
    vel = np.zeros((3, 9))
    vel[1, 6] = 1e3  # the pair at x = 9 flies apart
    mass = np.full(9, 0.1)
    label, cl, members, pairs = orc.groups(pos, vel, mass, r_in, theta)
    assert list(label) == [0, 0, 0, 3, 3, 5, 5, 7, 7]
    assert list(np.diff(cl)) == [3, 2, 2, 2]
    assert pairs.tolist() == [[3, 4], [7, 8]]
    # the relation itself against the definition, pair by pair
    offs, idx = orc.group_relation(pos, r_in, theta)
    for i in range(9):
        want = [j for j in range(9) if j != i and
                np.linalg.norm(pos[:, j] - pos[:, i]) < theta * max(r_in[i], r_in[j])]
        assert list(idx[offs[i]:offs[i + 1]]) == want


def test_groups_match_bfs(orc):
    """Random clustered points: components by breadth-first search over the
    brute-force relation written out in numpy."""
    rng = np.random.default_rng(21)
    n = 300
    pos = rng.uniform(0, 1, (3, n))
    pos[:, 150:] = pos[:, :150] + rng.normal(scale=0.004, size=(3, 150))
    r_in = rng.uniform(0.004, 0.02, n)
    theta = 0.7
    label, cl, members, pairs = orc.groups(pos, np.zeros((3, n)), np.full(n, 1e-3), r_in, theta)
    d = np.linalg.norm(pos[:, :, None] - pos[:, None, :], axis=0)
    adj = (d < theta * np.maximum(r_in[:, None], r_in[None, :])) & ~np.eye(n, dtype=bool)
    want = np.full(n, -1)
    for s in range(n):
        if want[s] >= 0:
            continue
        comp, todo = [s], [s]
        want[s] = s
        while todo:
            u = todo.pop()
            for v in np.nonzero(adj[u])[0]:
                if want[v] < 0:
                    want[v] = s
                    todo.append(v)
    assert np.array_equal(label, want)
    sizes = np.bincount(want, minlength=n)
    assert sorted(map(tuple, pairs.tolist())) == sorted(
        (s, int(np.nonzero(want == s)[0][1])) for s in range(n) if sizes[s] == 2)


def test_kick_is_exact_on_dyadic_values(orc):
    v = np.array([[0.5, -0.75], [1.0, 0.0], [0.125, 3.0]])
    a = np.array([[0.25, 1.0], [-2.0, 4.0], [0.0, -0.5]])
    out = orc.kick(v, a, 2.0 ** -8)
    assert np.array_equal(out, v + a / 256.0)
    assert np.array_equal(orc.kick(out, a, -(2.0 ** -8)), v)


def test_kick_drives_a_kepler_orbit(orc):
    """The kick is pinned by the mechanics it serves: a kick-drift-kick
    integration whose kicks are oracle.kick with the long-range field of the
    direct sum (the pair stays beyond r_out, so the field is Newtonian)
    carries two equal masses around their circular orbit. The separation
    stays 1 and after one period 2 pi sqrt(a^3 / (G M)) both bodies are back
    at their start, within the O(dt^2) phase error of the leapfrog. A kick
    with the wrong sign, without dt or with the full step breaks the orbit."""
    pos = np.array([[0.5, -0.5], [0.0, 0.0], [0.0, 0.0]])
    vel = np.array([[0.0, 0.0], [0.5, -0.5], [0.0, 0.0]])
    mass = np.array([0.5, 0.5])
    r_in, r_out = np.full(2, 0.01), np.full(2, 0.1)
    steps = 2000
    dt = 2.0 * math.pi / steps
    start = pos.copy()
    acc, _ = orc.force_long(pos, mass, r_in, r_out)
    worst = 0.0
    for _ in range(steps):
        vel = orc.kick(vel, acc, 0.5 * dt)
        pos = pos + vel * dt
        acc, _ = orc.force_long(pos, mass, r_in, r_out)
        vel = orc.kick(vel, acc, 0.5 * dt)
        worst = max(worst, abs(np.linalg.norm(pos[:, 0] - pos[:, 1]) - 1.0))
    assert worst < 2e-5, worst
    assert np.abs(pos - start).max() < 1e-4, np.abs(pos - start).max()


def test_binaries_near_zero_energy(orc):
    """Pairs within a few ulp of zero Kepler energy: the oracle's bound
    binaries are the pairs whose energy, rounded as written, is negative;
    evaluating the squares with fused multiply-adds flips some of them, so
    the same set pins the GPU's decision to the unfused rounding."""
    from critical_pairs import fused_signs, near_zero_energy_pairs
    pos, vel, mass = near_zero_energy_pairs(1500, 3)
    n = pos.shape[1]
    _, _, _, pairs = orc.groups(pos, vel, mass, np.full(n, 0.01), 0.5)
    want = []
    for b in range(n // 2):
        r = pos[:, 2 * b + 1] - pos[:, 2 * b]
        v = vel[:, 2 * b + 1] - vel[:, 2 * b]
        rr = math.sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2])
        E = 0.5 * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]) - (mass[2 * b] + mass[2 * b + 1]) / rr
        if E < 0.0:
            want.append((2 * b, 2 * b + 1))
    assert pairs.tolist() == [list(p) for p in want]
    flipped = fused_signs(pos, vel, mass) != np.isin(np.arange(n // 2), [p[0] // 2 for p in want])
    assert flipped.sum() >= 10, flipped.sum()
