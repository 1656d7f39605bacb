"""FP64 CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package. The product library never calls
it, and it shares no code with the GPU path: ``oracle.c`` is a separate
implementation of the paper's definitions, compiled by gcc.

Every function cites the passage of the PeTar paper (Wang et al. 2020) it
follows; see ``oracle.c`` for the formulas. Parity status per function:
  changeover f/W/K, radii, direct long/short/Newton sums, neighbour lists,
  multipole field: pinned by the tests in ``tests/test_oracle_pins.py``.
  Kepler pericentre, second-stage neighbour filter and clusters: pinned by
  closed-form orbits and brute-force components.
  tidal-tensor fit and pseudoparticles: pinned by the closed forms of the
  paper's Table A, its condition numbers, exact recovery of polynomial
  fields, Taylor limits of a point-mass field and eq. avebinquad.
  tree force at theta > 0: pinned at theta = 0 (equals the direct sum) and by
  the multipole error law; its absolute truncation error at theta > 0 is
  measured only ("parity unpinned" by the paper, which prints no force-error
  numbers).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_i64_p = ctypes.POINTER(ctypes.c_int64)
_c_i32_p = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (-O2, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        d, i64, i32, p_d, p_i64, p_i32 = (ctypes.c_double, ctypes.c_int64, ctypes.c_int32,
                                         _c_double_p, _c_i64_p, _c_i32_p)
        for name in ("oracle_f", "oracle_W", "oracle_K"):
            fn = getattr(L, name)
            fn.argtypes = [d, d]
            fn.restype = d
        L.oracle_radii.argtypes = [p_d, p_d, i64, d, d, d, d, p_d, p_d, p_d]
        L.oracle_radii.restype = ctypes.c_int
        for name in ("oracle_force_long", "oracle_force_short"):
            fn = getattr(L, name)
            fn.argtypes = [p_d, p_d, p_d, p_d, i64, d, p_i64, i64, p_d, p_d]
            fn.restype = None
        L.oracle_force_newton.argtypes = [p_d, p_d, i64, d, p_i64, i64, p_d, p_d]
        L.oracle_force_newton.restype = None
        L.oracle_neighbours.argtypes = [p_d, p_d, i64, p_i64, i64, p_i64, p_i32, i64]
        L.oracle_neighbours.restype = i64
        L.oracle_multipole.argtypes = [p_d, p_d, i64, p_d, p_d, p_d]
        L.oracle_multipole.restype = None
        L.oracle_multipole_eval.argtypes = [d, p_d, p_d, d, p_d, i64, p_d, p_d]
        L.oracle_multipole_eval.restype = None
        L.oracle_tree_info.argtypes = [p_d, p_d, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       p_i64]
        L.oracle_tree_info.restype = ctypes.c_int
        L.oracle_tree_force.argtypes = [p_d, p_d, p_d, p_d, p_d, i64, d, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int, d, p_i64, i64, ctypes.c_int,
                                        p_d, p_d, p_i64]
        L.oracle_tree_force.restype = ctypes.c_int
        L.oracle_pericentre.argtypes = [p_d, p_d, d, p_d, p_d, d, d]
        L.oracle_pericentre.restype = d
        L.oracle_nb_filter.argtypes = [p_d, p_d, p_d, p_d, i64, d, d, p_i64, p_i32, p_i64, p_i32,
                                       i64]
        L.oracle_nb_filter.restype = i64
        L.oracle_clusters.argtypes = [i64, p_i64, p_i32, p_i32, p_i64, p_i32]
        L.oracle_clusters.restype = i64
        L.oracle_tidal_points.argtypes = [ctypes.c_int, p_d, d, p_d]
        L.oracle_tidal_points.restype = ctypes.c_int
        L.oracle_tidal_ginv.argtypes = [ctypes.c_int, p_d]
        L.oracle_tidal_ginv.restype = ctypes.c_int
        L.oracle_tidal_fit.argtypes = [ctypes.c_int, d, p_d, p_d, p_d]
        L.oracle_tidal_fit.restype = ctypes.c_int
        L.oracle_tidal_eval.argtypes = [ctypes.c_int, p_d, p_d, d, p_d, p_d]
        L.oracle_tidal_eval.restype = None
        L.oracle_pseudo_particles.argtypes = [d, d, p_d, p_d, p_d, p_d, d, p_d, p_d]
        L.oracle_group_relation.argtypes = [p_d, p_d, i64, d, p_i64, p_i32, i64]
        L.oracle_group_relation.restype = i64
        L.oracle_binary_elements.argtypes = [d, d, p_d, p_d, p_d, p_d, d, p_d]
        L.oracle_binary_elements.restype = ctypes.c_int
        L.oracle_pseudo_particles.restype = ctypes.c_int
        _lib = L
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a: Optional[np.ndarray], t=_c_double_p):
    return None if a is None else a.ctypes.data_as(t)


# ---------------------------------------------------------------- changeover
def f(x: float, lam: float) -> float:
    """f(x) of the mass-dependent changeover section."""
    return lib().oracle_f(float(x), float(lam))


def W(x: float, lam: float) -> float:
    """Potential changeover weight W(x)."""
    return lib().oracle_W(float(x), float(lam))


def K(x: float, lam: float) -> float:
    """Force changeover weight K(x) (eq. Wij)."""
    return lib().oracle_K(float(x), float(lam))


# --------------------------------------------------------------------- radii
def radii(mass, r_in_ref: float, r_out_ref: float, search_factor: float = 1.2,
          vel=None, cr_dt: float = 0.0):
    """(r_in, r_out, r_search) per particle: eq. rcut, then search_factor*r_out
    or eq. rnb (r_out + C_r |v| dt_L, with cr_dt = C_r dt_L) if vel is given."""
    m = _f64(mass)
    n = m.size
    v = None if vel is None else _f64(vel)
    rin, rout, rs = np.empty(n), np.empty(n), np.empty(n)
    rc = lib().oracle_radii(_p(m), _p(v), n, r_in_ref, r_out_ref, search_factor, cr_dt,
                            _p(rin), _p(rout), _p(rs))
    if rc != 0:
        raise ValueError("invalid radii arguments")
    return rin, rout, rs


# --------------------------------------------------------------- direct sums
def _targets(n, idx):
    if idx is None:
        return None, n
    ix = np.ascontiguousarray(idx, dtype=np.int64)
    return ix, ix.size


def force_long(pos, mass, r_in, r_out, G: float = 1.0, idx=None):
    """Direct-sum long-range acceleration (3, k) and potential (k,) (H_L of eq. cf)."""
    pos, mass, r_in, r_out = _f64(pos), _f64(mass), _f64(r_in), _f64(r_out)
    n = mass.size
    ix, k = _targets(n, idx)
    acc, pot = np.empty((3, k)), np.empty(k)
    lib().oracle_force_long(_p(pos), _p(mass), _p(r_in), _p(r_out), n, G, _p(ix, _c_i64_p), k,
                            _p(acc), _p(pot))
    return acc, pot


def force_short(pos, mass, r_in, r_out, G: float = 1.0, idx=None):
    """Direct-sum short-range companion (H_S of eq. cf)."""
    pos, mass, r_in, r_out = _f64(pos), _f64(mass), _f64(r_in), _f64(r_out)
    n = mass.size
    ix, k = _targets(n, idx)
    acc, pot = np.empty((3, k)), np.empty(k)
    lib().oracle_force_short(_p(pos), _p(mass), _p(r_in), _p(r_out), n, G, _p(ix, _c_i64_p), k,
                             _p(acc), _p(pot))
    return acc, pot


def force_newton(pos, mass, G: float = 1.0, idx=None):
    """Plain Newtonian direct sum."""
    pos, mass = _f64(pos), _f64(mass)
    n = mass.size
    ix, k = _targets(n, idx)
    acc, pot = np.empty((3, k)), np.empty(k)
    lib().oracle_force_newton(_p(pos), _p(mass), n, G, _p(ix, _c_i64_p), k, _p(acc), _p(pot))
    return acc, pot


def neighbours(pos, r_search, idx=None):
    """Neighbour candidates as CSR (offsets int64 [k+1], indices int32), ascending j."""
    pos, rs = _f64(pos), _f64(r_search)
    n = rs.size
    ix, k = _targets(n, idx)
    counts = np.empty(k, dtype=np.int64)
    total = lib().oracle_neighbours(_p(pos), _p(rs), n, _p(ix, _c_i64_p), k,
                                    _p(counts, _c_i64_p), None, 0)
    out = np.empty(max(total, 1), dtype=np.int32)
    lib().oracle_neighbours(_p(pos), _p(rs), n, _p(ix, _c_i64_p), k, _p(counts, _c_i64_p),
                            _p(out, _c_i32_p), out.size)
    offs = np.zeros(k + 1, dtype=np.int64)
    offs[1:] = np.cumsum(counts)
    return offs, out[:total]


# ---------------------------------------------------------------- multipoles
def multipole(pos, mass):
    """(M, com[3], quad6) about the centre of mass (eq. quad, eq. quadtr)."""
    pos, mass = _f64(pos), _f64(mass)
    M = ctypes.c_double()
    com, q = np.empty(3), np.empty(6)
    lib().oracle_multipole(_p(pos), _p(mass), mass.size, ctypes.byref(M), _p(com), _p(q))
    return M.value, com, q


def multipole_eval(M, com, quad6, pts, G: float = 1.0):
    pts = _f64(pts)
    npts = pts.shape[1]
    acc, pot = np.empty((3, npts)), np.empty(npts)
    lib().oracle_multipole_eval(float(M), _p(_f64(com)), _p(_f64(quad6)), G, _p(pts), npts,
                                _p(acc), _p(pot))
    return acc, pot


# ---------------------------------------------------------------------- tree
def tree_info(pos, mass, leaf_size: int, group_size: int, max_level: int = 21) -> dict:
    pos, mass = _f64(pos), _f64(mass)
    info = np.zeros(6, dtype=np.int64)
    rc = lib().oracle_tree_info(_p(pos), _p(mass), mass.size, leaf_size, group_size, max_level,
                                _p(info, _c_i64_p))
    if rc != 0:
        raise ValueError("invalid tree arguments")
    keys = ("n_cells", "n_leaves", "n_groups", "max_level", "max_leaf", "sum_leaf")
    return {k: int(v) for k, v in zip(keys, info)}


def tree_force(pos, mass, r_in, r_out, r_search, theta: float, leaf_size: int,
               group_size: int, G: float = 1.0, idx=None, max_level: int = 21,
               skip_massless: bool = False):
    """Barnes-Hut long-range force with the group-wise walk (tree depth
    max_level: 21 for a single system, 18 per system in batched mode).
    skip_massless: the walk drops cells of zero mass and the leaf lists
    particles of zero mass (the rule of a force on a subset of targets),
    which changes the counts but no value.

    Returns (acc (3,k), pot (k,), counts (4,k)) where counts rows are:
    multipole cells, far-leaf particles, near-leaf particles, group size.
    """
    pos, mass = _f64(pos), _f64(mass)
    r_in, r_out, r_search = _f64(r_in), _f64(r_out), _f64(r_search)
    n = mass.size
    ix, k = _targets(n, idx)
    acc, pot = np.empty((3, k)), np.empty(k)
    counts = np.empty((4, k), dtype=np.int64)
    rc = lib().oracle_tree_force(_p(pos), _p(mass), _p(r_in), _p(r_out), _p(r_search), n,
                                 float(theta), int(leaf_size), int(group_size),
                                 int(max_level), G,
                                 _p(ix, _c_i64_p), k, int(bool(skip_massless)), _p(acc), _p(pot),
                                 _p(counts, _c_i64_p))
    if rc != 0:
        raise ValueError("invalid tree arguments")
    return acc, pot, counts


# ------------------------------------------------- second stage and clusters
def pericentre(xi, vi, mi: float, xj, vj, mj: float, G: float = 1.0) -> float:
    """Pericentre separation of the two-body Kepler orbit of a pair (Sec.
    "Orbit-dependent neighbour criterion", second stage)."""
    return lib().oracle_pericentre(_p(_f64(xi)), _p(_f64(vi)), float(mi), _p(_f64(xj)),
                                   _p(_f64(vj)), float(mj), float(G))


def nb_filter(pos, vel, mass, r_nb, c_v: float, offsets, idx, G: float = 1.0):
    """True neighbours among the candidate CSR: r_p,ij < c_v * r_nb,i."""
    pos, vel, mass, r_nb = _f64(pos), _f64(vel), _f64(mass), _f64(r_nb)
    n = mass.size
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    counts = np.empty(n, dtype=np.int64)
    out = np.empty(max(idx.size, 1), dtype=np.int32)
    total = lib().oracle_nb_filter(_p(pos), _p(vel), _p(mass), _p(r_nb), n, float(c_v), float(G),
                                   _p(offsets, _c_i64_p), _p(idx, _c_i32_p),
                                   _p(counts, _c_i64_p), _p(out, _c_i32_p), out.size)
    offs = np.zeros(n + 1, dtype=np.int64)
    offs[1:] = np.cumsum(counts)
    return offs, out[:total]


def clusters(n: int, offsets, idx):
    """Connected components of the neighbour graph (Sec. "Clustering"):
    (label int32 [n] = smallest member index, cluster offsets int64
    [n_clusters + 1], members int32 [n]), clusters by label, members
    ascending."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    label = np.empty(n, dtype=np.int32)
    cl = np.empty(n + 1, dtype=np.int64)
    members = np.empty(n, dtype=np.int32)
    nc = lib().oracle_clusters(int(n), _p(offsets, _c_i64_p), _p(idx, _c_i32_p),
                               _p(label, _c_i32_p), _p(cl, _c_i64_p), _p(members, _c_i32_p))
    return label, cl[:nc + 1].copy(), members


# --------------------------------------------------- artificial particles
def tidal_points(order: int, cm, d_c: float) -> np.ndarray:
    """Measure points (P, 3) of the order-2 (tetrahedron) or order-3 tidal
    tensor around cm (Table A)."""
    P = 4 if order == 2 else 8
    out = np.empty(3 * P)
    if lib().oracle_tidal_points(int(order), _p(_f64(cm)), float(d_c), _p(out)) != P:
        raise ValueError("order must be 2 or 3")
    return out.reshape(P, 3)


def tidal_ginv(order: int) -> np.ndarray:
    """Generalized inverse (K, 3P) of the measure-point map for d_c = 1
    (eq. map)."""
    K, P = (6, 4) if order == 2 else (16, 8)
    out = np.empty(K * 3 * P)
    if lib().oracle_tidal_ginv(int(order), _p(out)) != K:
        raise ValueError("bad order or rank-deficient map")
    return out.reshape(K, 3 * P)


def tidal_fit(order: int, d_c: float, acc_cm, acc_pts) -> np.ndarray:
    """[A(r_cm) (3), tensor coefficients (6 or 16)] from the accelerations
    at the centre and at the measure points (P, 3)."""
    K = 6 if order == 2 else 16
    out = np.empty(3 + K)
    rc = lib().oracle_tidal_fit(int(order), float(d_c), _p(_f64(acc_cm)),
                                _p(_f64(np.asarray(acc_pts).reshape(-1))), _p(out))
    if rc != 3 + K:
        raise ValueError("tidal fit failed")
    return out


def tidal_eval(order: int, t, rp) -> np.ndarray:
    """Field of the fitted model t = [A(r_cm), T] at offset rp from the
    centre (the evaluation rows of Table A)."""
    out = np.empty(3)
    lib().oracle_tidal_eval(int(order), _p(_f64(t)), _p(_f64(rp)), 0.0, _p(out), None)
    return out


def tidal_potential(order: int, t, rp, phi_cm: float) -> float:
    """Potential of the fitted model (minus its gradient is tidal_eval)."""
    out = np.empty(3)
    pot = ctypes.c_double()
    lib().oracle_tidal_eval(int(order), _p(_f64(t)), _p(_f64(rp)), float(phi_cm), _p(out),
                            ctypes.byref(pot))
    return pot.value


def binary_elements(m1, m2, x1, x2, v1, v2, G: float = 1.0):
    """(a, e) of a bound two-body orbit, or None when unbound."""
    out = np.empty(2)
    rc = lib().oracle_binary_elements(float(m1), float(m2), _p(_f64(x1)), _p(_f64(x2)),
                                      _p(_f64(v1)), _p(_f64(v2)), float(G), _p(out))
    return None if rc != 0 else (float(out[0]), float(out[1]))


def pseudo_particles(m1, m2, x1, x2, v1, v2, G: float = 1.0):
    """Positions (3, 3) and common mass of the three pseudoparticles of a
    bound binary (eq. psep, rotated into the orbit's frame), or None for an
    unbound or degenerate pair."""
    pos = np.empty(9)
    m = ctypes.c_double()
    rc = lib().oracle_pseudo_particles(float(m1), float(m2), _p(_f64(x1)), _p(_f64(x2)),
                                       _p(_f64(v1)), _p(_f64(v2)), float(G), _p(pos),
                                       ctypes.byref(m))
    if rc != 0:
        return None
    return pos.reshape(3, 3), m.value


def artificial_set(pos, vel, mass, r_in, r_out, r_search, pairs, order: int, c_d: float,
                   G: float = 1.0) -> dict:
    """Particle set of the long-range force with artificial particles (Sec.
    "Artificial particle algorithm for weak perturbation"; the cycle of
    Sec. "Implementation", where the tree of the long-range step includes
    the artificial particles).

    pos, vel (3, N); mass, radii (N,); pairs (n_pair, 2) input indices of
    bound binaries. The members of the pairs are left out; the singles come
    first in input order, then one block per pair: its centre of mass and
    the P measure points of Table A (zero mass) and the three
    pseudoparticles of eq. psep (mass (m1 + m2)/3 each). Every artificial
    particle takes the larger of the members' radii; d_c = c_d a (1 + e).
    Returns dict(pos (3, n_out), mass, r_in, r_out, r_search, src (n_out,),
    -1 for artificial particles), frame (n_pair, 4) = (r_cm, d_c), pair_of
    (N,), n_single). Raises ValueError for an unbound pair or a particle in
    two pairs.
    """
    pos = np.asarray(pos, dtype=np.float64)
    vel = np.asarray(vel, dtype=np.float64)
    n = pos.shape[1]
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    P = 4 if order == 2 else 8
    pair_of = np.full(n, -1, dtype=np.int64)
    for b, (i, j) in enumerate(pairs):
        if i == j or pair_of[i] >= 0 or pair_of[j] >= 0:
            raise ValueError("a particle in two pairs")
        pair_of[i] = pair_of[j] = b
    singles = np.nonzero(pair_of < 0)[0]
    n_s, n_p = len(singles), len(pairs)
    n_out = n_s + n_p * (P + 4)
    out = dict(pos=np.zeros((3, n_out)), mass=np.zeros(n_out), r_in=np.zeros(n_out),
               r_out=np.zeros(n_out), r_search=np.zeros(n_out),
               src=np.full(n_out, -1, dtype=np.int64), frame=np.zeros((n_p, 4)),
               pair_of=pair_of, n_single=n_s)
    out["pos"][:, :n_s] = pos[:, singles]
    out["mass"][:n_s] = mass[singles]
    for name, arr in (("r_in", r_in), ("r_out", r_out), ("r_search", r_search)):
        out[name][:n_s] = np.asarray(arr)[singles]
    out["src"][:n_s] = singles
    for b, (i, j) in enumerate(pairs):
        m1, m2 = float(mass[i]), float(mass[j])
        el = binary_elements(m1, m2, pos[:, i], pos[:, j], vel[:, i], vel[:, j], G)
        pp = pseudo_particles(m1, m2, pos[:, i], pos[:, j], vel[:, i], vel[:, j], G)
        if el is None or pp is None:
            raise ValueError("pair %d is not bound" % b)
        a, e = el
        cm = (m1 * pos[:, i] + m2 * pos[:, j]) / (m1 + m2)
        d_c = c_d * a * (1.0 + e)
        out["frame"][b] = (*cm, d_c)
        base = n_s + b * (P + 4)
        out["pos"][:, base] = cm
        out["pos"][:, base + 1:base + 1 + P] = tidal_points(order, cm, d_c).T
        out["pos"][:, base + 1 + P:base + 4 + P] = pp[0].T
        out["mass"][base + 1 + P:base + 4 + P] = pp[1]
        for name, arr in (("r_in", r_in), ("r_out", r_out), ("r_search", r_search)):
            out[name][base:base + P + 4] = max(float(arr[i]), float(arr[j]))
    return out


def artificial_fit(order: int, art: dict, pos, acc_set, pot_set, pairs):
    """Post-fit of the long-range step: per pair the record [phi(r_cm),
    A(r_cm), T] from the accelerations (and potentials) of its centre and
    measure points; per input particle the long-range acceleration and
    potential: singles take theirs from the set, members the fitted field
    at their position.
    acc_set (3, n_out), pot_set (n_out,). Returns (records (n_pair, 4 + K),
    acc (3, N), pot (N,))."""
    P = 4 if order == 2 else 8
    K = 6 if order == 2 else 16
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[1]
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    n_s = art["n_single"]
    rec = np.zeros((len(pairs), 4 + K))
    acc = np.zeros((3, n))
    pot = np.zeros(n)
    src = art["src"][:n_s]
    acc[:, src] = acc_set[:, :n_s]
    pot[src] = pot_set[:n_s]
    for b, (i, j) in enumerate(pairs):
        base = n_s + b * (P + 4)
        cm, d_c = art["frame"][b, :3], art["frame"][b, 3]
        t = tidal_fit(order, d_c, acc_set[:, base], acc_set[:, base + 1:base + 1 + P].T)
        rec[b, 0] = pot_set[base]
        rec[b, 1:] = t
        for m in (i, j):
            rp = pos[:, m] - cm
            acc[:, m] = tidal_eval(order, t, rp)
            pot[m] = tidal_potential(order, t, rp, pot_set[base])
    return rec, acc, pot


# ------------------------------------------------------------ SDAR groups
def group_relation(pos, r_in, theta: float):
    """CSR (offsets int64 [N+1], idx int32) of the pairs r_ij < theta
    r_in,ij (eq. rbin), all j != i ascending, by brute force."""
    pos, r_in = _f64(pos), _f64(r_in)
    n = r_in.size
    counts = np.empty(n, dtype=np.int64)
    total = lib().oracle_group_relation(_p(pos), _p(r_in), n, float(theta), _p(counts, _c_i64_p),
                                        None, 0)
    out = np.empty(max(total, 1), dtype=np.int32)
    lib().oracle_group_relation(_p(pos), _p(r_in), n, float(theta), _p(counts, _c_i64_p),
                                _p(out, _c_i32_p), out.size)
    offs = np.zeros(n + 1, dtype=np.int64)
    offs[1:] = np.cumsum(counts)
    return offs, out[:total]


def groups(pos, vel, mass, r_in, theta: float, G: float = 1.0):
    """SDAR groups (Sec. "SDAR", eq. rbin): (label, offsets, members) as
    clusters() of the pair relation r_ij < theta r_in,ij, and the bound
    binaries (n_pairs, 2): the groups of exactly two members with negative
    Kepler energy, in group order, smaller index first."""
    offs, idx = group_relation(pos, r_in, theta)
    label, cl, members = clusters(len(r_in), offs, idx)
    pos, vel = np.asarray(pos), np.asarray(vel)
    pairs = []
    for g in range(len(cl) - 1):
        if cl[g + 1] - cl[g] != 2:
            continue
        i, j = int(members[cl[g]]), int(members[cl[g] + 1])
        if binary_elements(mass[i], mass[j], pos[:, i], pos[:, j], vel[:, i], vel[:, j],
                           G) is not None:
            pairs.append((i, j))
    return label, cl, members, np.array(pairs, dtype=np.int64).reshape(-1, 2)


def kick(vel, acc, dt: float):
    """Velocity kick of the long-range step, v + a_L dt (eq. lfmap with dt
    the half step of the KDK cycle)."""
    return np.asarray(vel, dtype=np.float64) + np.asarray(acc, dtype=np.float64) * dt
