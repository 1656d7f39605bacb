"""Pairs whose Kepler energy (eq. dr) lies within a few ulp of zero.

Which of them count as bound is decided by the last bit of the FP64
arithmetic, so they pin that the decision is rounded exactly as written
(squares summed x, y, then z; no fused multiply-add). `fused_signs`
evaluates the same energies with the squares accumulated by fused
multiply-adds, to show that the set tells the two apart.
"""

from fractions import Fraction

import numpy as np


def near_zero_energy_pairs(k: int, seed: int):
    """k pairs 10 length units apart along x, separation ~1e-3 in a random
    direction, relative speed sqrt(2 G (m_i + m_j) / r) times (1 + d) with
    |d| below a few ulp. Returns pos [3, 2k], vel [3, 2k], mass [2k]."""
    rng = np.random.default_rng(seed)
    pos = np.zeros((3, 2 * k))
    vel = np.zeros((3, 2 * k))
    mass = rng.uniform(1e-6, 1e-4, 2 * k)
    for b in range(k):
        i, j = 2 * b, 2 * b + 1
        pos[:, i] = (10.0 * b, 0.0, 0.0)
        u = rng.normal(size=3)
        pos[:, j] = pos[:, i] + 1e-3 * rng.uniform(0.5, 1.5) * u / np.linalg.norm(u)
        r = pos[:, j] - pos[:, i]
        rr = np.sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2])
        w = rng.normal(size=3)
        speed = np.sqrt(2.0 * (mass[i] + mass[j]) / rr) * (1.0 + rng.uniform(-4, 4) * 2.0 ** -53)
        vel[:, i] = rng.normal(size=3) * 1e-2
        vel[:, j] = vel[:, i] + speed * w / np.linalg.norm(w)
    return pos, vel, mass


def _fma(a: float, b: float, c: float) -> float:
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def fused_signs(pos, vel, mass, G: float = 1.0):
    """Bound flags of the pairs (2b, 2b + 1) with the squared separation and
    speed accumulated as fma(z, z, fma(y, y, x * x)); the rest as written."""
    out = []
    for b in range(pos.shape[1] // 2):
        i, j = 2 * b, 2 * b + 1
        r = pos[:, j] - pos[:, i]
        v = vel[:, j] - vel[:, i]
        r2 = _fma(r[2], r[2], _fma(r[1], r[1], r[0] * r[0]))
        v2 = _fma(v[2], v[2], _fma(v[1], v[1], v[0] * v[0]))
        rr = np.sqrt(r2)
        E = 0.5 * v2 - G * (mass[i] + mass[j]) / rr
        out.append(bool(rr > 0.0 and E < 0.0))
    return np.array(out)
