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
                                        ctypes.c_int, ctypes.c_int, d, p_i64, i64, p_d, p_d,
                                        p_i64]
        L.oracle_tree_force.restype = ctypes.c_int
        L.oracle_pericentre.argtypes = [p_d, p_d, d, p_d, p_d, d, d]
        L.oracle_pericentre.restype = d
        L.oracle_nb_filter.argtypes = [p_d, p_d, p_d, p_d, i64, d, d, p_i64, p_i32, p_i64, p_i32,
                                       i64]
        L.oracle_nb_filter.restype = i64
        L.oracle_clusters.argtypes = [i64, p_i64, p_i32, p_i32, p_i64, p_i32]
        L.oracle_clusters.restype = i64
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
               group_size: int, G: float = 1.0, idx=None, max_level: int = 21):
    """Barnes-Hut long-range force with the group-wise walk (tree depth
    max_level: 21 for a single system, 18 per system in batched mode).

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
                                 _p(ix, _c_i64_p), k, _p(acc), _p(pot), _p(counts, _c_i64_p))
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
