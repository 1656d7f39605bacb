"""Seeded synthetic star-cluster inputs (test and benchmark infrastructure).

This module only draws initial conditions. It holds none of the force
method's arithmetic: no changeover radii, no tree, no forces. Both the FP64
oracle and the GPU library are fed from here, so neither depends on the other.

Models follow the workloads of the PeTar paper (Sec. "Performance on
GPU-based Desktop"): a Plummer sphere in Henon (NB) units (G = M = 1,
virial radius 1), Kroupa (2001) IMF masses, and primordial binaries with
thermal eccentricities. The binary semi-major axes are drawn log-uniform in
a given range instead of the paper's Kroupa (1995) period law.

Methods used (published, restated here):
  * Plummer positions and velocities: Aarseth, Henon & Wielen (1974),
    A&A 37, 183 -- inverse of the cumulative mass M(<r) = r^3/(1+r^2)^{3/2}
    (a = 1) and von Neumann rejection on g(q) = q^2 (1-q^2)^{7/2}.
    Scaled to NB units by r -> r * 3*pi/16, v -> v * sqrt(16/(3*pi)).
  * Kroupa (2001) IMF: dN/dm ~ m^-1.3 on [0.08, 0.5) and m^-2.3 on
    [0.5, m_max], continuous at 0.5; inverse-CDF sampling per segment.
  * Binaries: Kepler orbit from (a, e, mean anomaly), solved for the
    eccentric anomaly by Newton iteration; isotropic orientation.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

PLUMMER_MASS_CUT = 0.999  # truncate the cumulative mass fraction (r < ~22.8 NB)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    """n unit vectors uniform on the sphere, shape (n, 3)."""
    cos_t = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    sin_t = np.sqrt(1.0 - cos_t * cos_t)
    return np.stack([sin_t * np.cos(phi), sin_t * np.sin(phi), cos_t], axis=1)


def plummer(rng: np.random.Generator, n: int) -> tuple[np.ndarray, np.ndarray]:
    """Positions and velocities (n, 3) of a Plummer sphere in NB units.

    Total mass 1 is assumed for the velocity scale (masses are set by the
    caller and sum to 1).
    """
    x = rng.uniform(0.0, PLUMMER_MASS_CUT, n)
    r = 1.0 / np.sqrt(x ** (-2.0 / 3.0) - 1.0)
    pos = r[:, None] * _isotropic(rng, n)
    # velocity modulus: q = v / v_esc with density g(q) = q^2 (1-q^2)^3.5
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        q_try = rng.uniform(0.0, 1.0, todo.size)
        y = rng.uniform(0.0, 0.1, todo.size)
        ok = y < q_try ** 2 * (1.0 - q_try ** 2) ** 3.5
        q[todo[ok]] = q_try[ok]
        todo = todo[~ok]
    v_esc = math.sqrt(2.0) * (1.0 + r * r) ** -0.25
    vel = (q * v_esc)[:, None] * _isotropic(rng, n)
    rscale = 3.0 * math.pi / 16.0
    return pos * rscale, vel / math.sqrt(rscale)


def kroupa_imf(rng: np.random.Generator, n: int, m_min: float = 0.08,
               m_max: float = 150.0) -> np.ndarray:
    """n masses (Msun) from the two-segment Kroupa (2001) IMF."""
    m_br = 0.5
    a1, a2 = 1.3, 2.3
    # segment integrals of k_s m^-a with continuity at m_br (k2 = k1 * m_br^(a2-a1))
    def seg_int(a, lo, hi):
        return (hi ** (1.0 - a) - lo ** (1.0 - a)) / (1.0 - a)
    lo1, hi1 = m_min, min(m_br, m_max)
    w1 = seg_int(a1, lo1, hi1) if hi1 > lo1 else 0.0
    lo2, hi2 = max(m_br, m_min), m_max
    w2 = m_br ** (a2 - a1) * seg_int(a2, lo2, hi2) if hi2 > lo2 else 0.0
    u_seg = rng.uniform(0.0, 1.0, n)
    u = rng.uniform(0.0, 1.0, n)
    in1 = u_seg < w1 / (w1 + w2)

    def inv(a, lo, hi, uu):
        return (lo ** (1.0 - a) + uu * (hi ** (1.0 - a) - lo ** (1.0 - a))) ** (1.0 / (1.0 - a))

    m = np.where(in1, inv(a1, lo1, hi1, u), inv(a2, lo2, hi2, u))
    return m


def _kepler_relative(rng: np.random.Generator, mtot: np.ndarray, a: np.ndarray,
                     e: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Relative position and velocity (n, 3) of Kepler orbits, G = 1."""
    n = a.size
    mean_anom = rng.uniform(0.0, 2.0 * math.pi, n)
    ecc_anom = mean_anom + e * np.sin(mean_anom)
    for _ in range(60):  # Newton on E - e sin E - M = 0
        f = ecc_anom - e * np.sin(ecc_anom) - mean_anom
        ecc_anom = ecc_anom - f / (1.0 - e * np.cos(ecc_anom))
    cos_e, sin_e = np.cos(ecc_anom), np.sin(ecc_anom)
    b = a * np.sqrt(1.0 - e * e)
    rel = np.stack([a * (cos_e - e), b * sin_e, np.zeros(n)], axis=1)
    n_mean = np.sqrt(mtot / a ** 3)
    edot = n_mean / (1.0 - e * cos_e)
    vrel = np.stack([-a * sin_e * edot, b * cos_e * edot, np.zeros(n)], axis=1)
    # random orientation: orthonormal frame from an isotropic normal
    z = _isotropic(rng, n)
    helper = np.where(np.abs(z[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    xax = np.cross(helper, z)
    xax /= np.linalg.norm(xax, axis=1, keepdims=True)
    psi = rng.uniform(0.0, 2.0 * math.pi, n)  # argument of pericentre
    yax = np.cross(z, xax)
    ex = np.cos(psi)[:, None] * xax + np.sin(psi)[:, None] * yax
    ey = -np.sin(psi)[:, None] * xax + np.cos(psi)[:, None] * yax
    pos = rel[:, :1] * ex + rel[:, 1:2] * ey
    vel = vrel[:, :1] * ex + vrel[:, 1:2] * ey
    return pos, vel


@dataclasses.dataclass(frozen=True)
class Cluster:
    pos: np.ndarray   # (3, N) float64, SoA
    vel: np.ndarray   # (3, N) float64, SoA
    mass: np.ndarray  # (N,) float64, sums to 1
    n_binaries: int
    pairs: np.ndarray = None  # (n_binaries, 2) int64: indices of the two members


def make_cluster(n: int, seed: int, *, imf: bool = True, binary_fraction: float = 0.0,
                 a_min: float = 1e-5, a_max: float = 1e-2, m_max: float = 150.0) -> Cluster:
    """A Plummer cluster of n stars in NB units.

    binary_fraction is the fraction of *stars* that are binary members
    (so n_binaries = round(binary_fraction * n / 2)). Binary components are
    two independent IMF draws placed about a Plummer-sampled centre of mass,
    with log-uniform a in [a_min, a_max], thermal e and random orientation.
    Without `imf` every star has mass 1/n exactly.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = _rng(seed)
    n_bin = int(round(binary_fraction * n / 2.0))
    n_bin = min(n_bin, n // 2)
    n_cm = n - n_bin
    if imf:
        m = kroupa_imf(rng, n, m_max=m_max)
        m = m / m.sum()
    else:
        m = np.full(n, 1.0 / n)
    pos_cm, vel_cm = plummer(rng, n_cm)
    pos = np.empty((n, 3))
    vel = np.empty((n, 3))
    n_single = n_cm - n_bin
    pos[:n_single] = pos_cm[:n_single]
    vel[:n_single] = vel_cm[:n_single]
    if n_bin:
        m1 = m[n_single:n_single + n_bin]
        m2 = m[n_single + n_bin:]
        mt = m1 + m2
        a = np.exp(rng.uniform(math.log(a_min), math.log(a_max), n_bin))
        e = np.sqrt(rng.uniform(0.0, 1.0, n_bin))
        drel, dvel = _kepler_relative(rng, mt, a, e)
        c_pos, c_vel = pos_cm[n_single:], vel_cm[n_single:]
        f1 = (m2 / mt)[:, None]
        f2 = (m1 / mt)[:, None]
        pos[n_single:n_single + n_bin] = c_pos - f1 * drel
        pos[n_single + n_bin:] = c_pos + f2 * drel
        vel[n_single:n_single + n_bin] = c_vel - f1 * dvel
        vel[n_single + n_bin:] = c_vel + f2 * dvel
    perm = rng.permutation(n)
    where = np.empty(n, dtype=np.int64)
    where[perm] = np.arange(n)
    pairs = np.stack([where[n_single:n_single + n_bin], where[n_single + n_bin:]], axis=1)
    return Cluster(pos=np.ascontiguousarray(pos[perm].T), vel=np.ascontiguousarray(vel[perm].T),
                   mass=np.ascontiguousarray(m[perm]), n_binaries=n_bin, pairs=pairs)


# --------------------------------------------------------------------------
# The five benchmark workloads (sizes and radii references).
# --------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int
    imf: bool
    binary_fraction: float
    theta: float
    leaf_size: int
    r_in_ref: float
    r_out_ref: float
    search_factor: float      # r_search,i = search_factor * r_out,i
    uniform_radii: bool       # equal masses: scalar radii, no mass factor


def r_out_ref_for(n: int) -> float:
    """Reference outer radius scaled as N^-1/3 from 0.02 at N = 65536."""
    return 0.02 * (65536.0 / n) ** (1.0 / 3.0)


WORKLOADS = {
    "plummer4k": Workload("plummer4k", 4096, False, 0.0, 0.5, 8, 0.01, 0.1, 1.2, True),
    "plummer64k_b50": Workload("plummer64k_b50", 65536, True, 0.5, 0.5, 8, 0.002, 0.02, 1.2, False),
    "plummer1m_b100": Workload("plummer1m_b100", 1048576, True, 1.0, 0.5, 8,
                               0.1 * r_out_ref_for(1048576), r_out_ref_for(1048576), 1.2, False),
    "plummer10m_b10": Workload("plummer10m_b10", 10485760, True, 0.1, 0.5, 8,
                               0.1 * r_out_ref_for(10485760), r_out_ref_for(10485760), 1.2, False),
}


def batched_sizes(seed: int, n_sys: int = 128, n_lo: int = 1024, n_hi: int = 131072) -> np.ndarray:
    """System sizes drawn log-uniformly in [n_lo, n_hi] (batched workload)."""
    rng = _rng(seed + 7919)
    return np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), n_sys))).astype(np.int64)


def make_batched(seed: int, n_sys: int = 128, binary_fraction: float = 0.2,
                 n_lo: int = 1024, n_hi: int = 131072):
    """n_sys independent clusters; returns (offsets[n_sys+1], pos(3,Ntot), vel, mass, sizes)."""
    sizes = batched_sizes(seed, n_sys, n_lo, n_hi)
    offs = np.zeros(n_sys + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)
    pos = np.empty((3, offs[-1]))
    vel = np.empty((3, offs[-1]))
    mass = np.empty(offs[-1])
    for k in range(n_sys):
        c = make_cluster(int(sizes[k]), seed * 1000003 + k, imf=True, binary_fraction=binary_fraction)
        pos[:, offs[k]:offs[k + 1]] = c.pos
        vel[:, offs[k]:offs[k + 1]] = c.vel
        mass[offs[k]:offs[k + 1]] = c.mass
    return offs, pos, vel, mass, sizes


def sample_indices(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct indices in [0, n), sorted, seeded (error subsample)."""
    if k >= n:
        return np.arange(n, dtype=np.int64)
    rng = _rng(seed + 104729)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)
