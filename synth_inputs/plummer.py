"""Plummer-sphere initial conditions in Henon N-body units.

The paper's tests use an equal-mass Plummer sphere in standard N-body units
(G = M = 1, E = -1/4, virial radius about 1; Plummer radius about 0.6 and
half-mass radius about 0.8), generated with an external tool that is not
available here (GraviDy paper, Sec. 3.1). This module stands in for it with the
classical Aarseth-Henon-Wielen (1974) sampling of the Plummer model:

* radius from the cumulative mass fraction X of the model with scale a = 1,
  r = (X^(-2/3) - 1)^(-1/2), with X drawn uniform on [0, 0.999) (the usual
  truncation of the far tail);
* isotropic directions for position and velocity;
* speed v = q * v_esc(r), v_esc = sqrt(2) (1 + r^2)^(-1/4), where q is drawn by
  von Neumann rejection from the density g(q) = q^2 (1 - q^2)^(7/2);
* centre-of-mass position and velocity removed;
* scaling from the a = 1 model (energy -3 pi / 64) to Henon units by the model's
  own constants: r <- r * 3 pi / 16, v <- v * sqrt(16 / (3 pi)).

The scaling is the model's, not the sample's: the sampled energy is -1/4 up to
the N^(-1/2) sampling noise (the paper's own example run starts at E0 = -0.256).

Every draw comes from numpy's PCG64 generator seeded by the caller, in a fixed
order, so a (N, seed) pair names a unique particle set.
"""
from __future__ import annotations

import math

import numpy as np

# Henon units for the Plummer model: G = M = 1, E = -1/4 (paper Sec. 3.1).
_LENGTH = 3.0 * math.pi / 16.0
_SPEED = math.sqrt(16.0 / (3.0 * math.pi))
_X_MAX = 0.999  # mass-fraction truncation of the radial tail


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    """n unit vectors uniform on the sphere (cos(theta) uniform, phi uniform)."""
    cth = 1.0 - 2.0 * rng.random(n)
    phi = 2.0 * math.pi * rng.random(n)
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    return np.stack([sth * np.cos(phi), sth * np.sin(phi), cth], axis=1)


def _speed_fraction(rng: np.random.Generator, n: int) -> np.ndarray:
    """q in [0, 1) with density proportional to q^2 (1 - q^2)^(7/2), by rejection.

    The density's maximum is about 0.092 (at q^2 = 2/9), so the envelope 0.1 is
    safe. Rejected candidates are redrawn in batches until n are accepted.
    """
    out = np.empty(n)
    filled = 0
    while filled < n:
        want = n - filled
        batch = max(64, int(want * 2.2))
        q = rng.random(batch)
        y = 0.1 * rng.random(batch)
        ok = q[y < q * q * (1.0 - q * q) ** 3.5]
        take = min(want, ok.size)
        out[filled:filled + take] = ok[:take]
        filled += take
    return out


def _plummer_xv(rng: np.random.Generator, n: int):
    """Positions and velocities of the a = 1, G = M = 1 Plummer model."""
    x_frac = _X_MAX * rng.random(n)
    # r = (X^(-2/3) - 1)^(-1/2); X = 0 maps to r = 0.
    with np.errstate(divide="ignore"):
        r = np.where(x_frac > 0.0, 1.0 / np.sqrt(np.power(x_frac, -2.0 / 3.0) - 1.0), 0.0)
    pos = r[:, None] * _isotropic(rng, n)
    q = _speed_fraction(rng, n)
    vesc = math.sqrt(2.0) * np.power(1.0 + r * r, -0.25)
    vel = (q * vesc)[:, None] * _isotropic(rng, n)
    return pos, vel


def _centre_and_scale(m: np.ndarray, pos: np.ndarray, vel: np.ndarray):
    msum = m.sum()
    pos = pos - (m[:, None] * pos).sum(axis=0) / msum
    vel = vel - (m[:, None] * vel).sum(axis=0) / msum
    return pos * _LENGTH, vel * _SPEED


def plummer(n: int, seed: int):
    """Equal-mass Plummer sphere: masses 1/n, Henon units.

    Returns (m[n], x[n, 3], v[n, 3]) as contiguous float64 arrays.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = np.random.Generator(np.random.PCG64(seed))
    pos, vel = _plummer_xv(rng, n)
    m = np.full(n, 1.0 / n)
    pos, vel = _centre_and_scale(m, pos, vel)
    return m, np.ascontiguousarray(pos), np.ascontiguousarray(vel)


def plummer_imf(n: int, seed: int, slope: float = -2.35, m_lo: float = 0.1, m_hi: float = 100.0):
    """Plummer positions and velocities with power-law masses dN/dm ~ m^slope.

    Masses by inverse CDF on [m_lo, m_hi], then normalised to a total of 1. The
    phase-space sample does not depend on the masses; the centre of mass is
    removed with the drawn masses.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = np.random.Generator(np.random.PCG64(seed))
    pos, vel = _plummer_xv(rng, n)
    p = slope + 1.0
    u = rng.random(n)
    lo, hi = m_lo ** p, m_hi ** p
    m = np.power(lo + u * (hi - lo), 1.0 / p)
    m = m / m.sum()
    pos, vel = _centre_and_scale(m, pos, vel)
    return m, np.ascontiguousarray(pos), np.ascontiguousarray(vel)


def plummer_with_bh(n_stars: int, seed: int, m_bh: float = 0.01):
    """Equal-mass Plummer stars (total mass 1) plus one massive particle at rest
    at the origin, stored last (index n_stars)."""
    m, x, v = plummer(n_stars, seed)
    m = np.concatenate([m, [m_bh]])
    x = np.concatenate([x, np.zeros((1, 3))])
    v = np.concatenate([v, np.zeros((1, 3))])
    return m, np.ascontiguousarray(x), np.ascontiguousarray(v)


def kepler_pair(m1: float = 0.5, m2: float = 0.5, a: float = 1.0, e: float = 0.0):
    """Two bodies on a bound Kepler orbit, started at pericentre, centre of mass
    at rest at the origin, orbit in the x-y plane (G = 1).

    Relative separation at pericentre a (1 - e); relative speed from the vis-viva
    relation sqrt(M (1 + e) / (a (1 - e))).
    """
    mt = m1 + m2
    rp = a * (1.0 - e)
    vp = math.sqrt(mt * (1.0 + e) / (a * (1.0 - e)))
    rel_x = np.array([rp, 0.0, 0.0])
    rel_v = np.array([0.0, vp, 0.0])
    x = np.stack([-m2 / mt * rel_x, m1 / mt * rel_x])
    v = np.stack([-m2 / mt * rel_v, m1 / mt * rel_v])
    return np.array([m1, m2]), x, v


# Workloads named by what they are (sizes, softening, step parameters).
WORKLOADS = {
    "plummer_n1024": dict(n=1024, seed=1, eps=1e-4, eta=0.01, dt_max=0.125, dt_min=2.0 ** -22, t_end=1.0),
    "plummer_n16384": dict(n=16384, seed=1, eps=1e-4, eta=0.01, dt_max=0.125, dt_min=2.0 ** -22, t_end=1.0),
    # power-law IMF (slope -2.35 on [0.1, 100], total mass 1): the mixed-precision workload
    "plummer_imf_n262144": dict(n=262144, seed=5, eps=1e-4, eta=0.01, dt_max=0.125, dt_min=2.0 ** -22,
                                t_end=0.125, imf=True),
    # 2^20 equal-mass stars plus a central particle of mass 0.01 at rest at the origin
    "plummer_bh_n1048576": dict(n=1048576 + 1, n_stars=1048576, seed=5, eps=1e-4, eps_bh=1e-6, m_bh=0.01,
                                eta=0.01, dt_max=0.125, dt_min=2.0 ** -22, t_end=0.125),
}
