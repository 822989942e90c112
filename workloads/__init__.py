"""Seeded synthetic initial conditions shared by the tests, the benchmark and
the oracle runs.

This module holds no part of the force method's arithmetic: it only draws
particle sets.  Every sampler works in FP64 with
``numpy.random.Generator(PCG64(seed))`` and casts at the end when an FP32
workload is asked for (round to nearest).

The paper's own initial conditions (a rotating stellar disc in equilibrium,
section 2) are described only qualitatively, so these recipes stand in for
them:
  * ``plummer`` — Plummer sphere, G = M = a = 1, truncated at r = 10 a by
    inverse-CDF sampling restricted to the truncated mass.
  * ``disc_galaxy`` — exponential disc (scale length 1, sech^2 height 0.1,
    truncated at R = 10) inside a Hernquist halo (scale radius 5, truncated
    at r = 100), with circular-velocity rotation plus Gaussian dispersion.
"""
from __future__ import annotations

import numpy as np

PLUMMER_RT = 10.0
PLUMMER_FT = PLUMMER_RT ** 3 / (PLUMMER_RT ** 2 + 1.0) ** 1.5  # M(<10)/M = 1000/101^1.5
DISC_ZT = 10.0  # sech^2 profile truncated at |z| = 10 z0


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _isotropic(g, r):
    n = r.shape[0]
    u = g.random((n, 2))
    cth = 2.0 * u[:, 0] - 1.0
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    ph = 2.0 * np.pi * u[:, 1]
    return np.stack([r * sth * np.cos(ph), r * sth * np.sin(ph), r * cth], axis=1)


def plummer(n: int, seed: int, dtype=np.float64, mass=None):
    """Plummer sphere (a = 1, total mass 1) truncated at r = 10.

    Returns (pos[n,3], mass[n]) in ``dtype``.  Masses are 1/n unless ``mass``
    gives another array.
    """
    g = rng(seed)
    U = g.random((n, 3))
    u = U[:, 0] * PLUMMER_FT
    u = np.maximum(u, 1e-300)
    r = 1.0 / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    cth = 2.0 * U[:, 1] - 1.0
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    ph = 2.0 * np.pi * U[:, 2]
    pos = np.stack([r * sth * np.cos(ph), r * sth * np.sin(ph), r * cth], axis=1)
    m = np.full(n, 1.0 / n) if mass is None else np.asarray(mass, np.float64)
    return pos.astype(dtype), m.astype(dtype)


def plummer_enclosed(r):
    """Truncated-Plummer M(<r) for the sampler above (total sampled mass 1)."""
    r = np.asarray(r, np.float64)
    return np.minimum(r ** 3 / (r * r + 1.0) ** 1.5 / PLUMMER_FT, 1.0)


def lognormal_masses(n: int, seed: int, sigma: float = 0.2):
    """m_i = (1/n) exp(sigma z - sigma^2/2), z ~ N(0,1): mean-preserving."""
    g = rng(seed)
    z = g.standard_normal(n)
    return np.exp(sigma * z - 0.5 * sigma * sigma) / n


def _disc_radius(g, n, Rt=10.0):
    # cumulative mass of an exponential disc: 1 - (1 + R) e^-R, solved by Newton
    Ft = 1.0 - (1.0 + Rt) * np.exp(-Rt)
    u = g.random(n) * Ft
    R = np.full(n, 1.5)
    for _ in range(60):
        f = 1.0 - (1.0 + R) * np.exp(-R) - u
        fp = R * np.exp(-R)
        R = np.clip(R - f / np.maximum(fp, 1e-300), 1e-12, Rt)
    return R


def disc_galaxy(n_disc: int, n_halo: int, seed: int, dtype=np.float32,
                m_disc_total: float = 1.0, m_halo_total: float = 4.0,
                halo_a: float = 5.0, halo_rt: float = 100.0, z0: float = 0.1):
    """Exponential disc + Hernquist halo.  Returns (pos, vel, mass)."""
    g = rng(seed)
    R = _disc_radius(g, n_disc)
    u = g.random(n_disc)
    z = z0 * np.arctanh((2.0 * u - 1.0) * np.tanh(DISC_ZT))
    ph = 2.0 * np.pi * g.random(n_disc)
    xd = np.stack([R * np.cos(ph), R * np.sin(ph), z], axis=1)
    # Hernquist halo truncated at halo_rt: M(<r) ∝ r^2/(r+a)^2
    c = (halo_rt / (halo_rt + halo_a)) ** 2
    X = g.random(n_halo) * c
    sX = np.sqrt(X)
    rh = halo_a * sX / (1.0 - sX)
    xh = _isotropic(g, rh)
    # velocities: disc on circular orbits plus dispersion, halo isotropic
    Md = m_disc_total * (1.0 - (1.0 + R) * np.exp(-R))
    Mh_R = m_halo_total * R * R / (R + halo_a) ** 2 / c
    vc = np.sqrt(np.maximum(Md + Mh_R, 0.0) / np.maximum(R, 1e-12))
    sig = np.stack([0.1 * vc, 0.1 * vc, 0.05 * vc], axis=1) * g.standard_normal((n_disc, 3))
    vR, vphi, vz = sig[:, 0], vc + sig[:, 1], sig[:, 2]
    vd = np.stack([vR * np.cos(ph) - vphi * np.sin(ph), vR * np.sin(ph) + vphi * np.cos(ph), vz], axis=1)
    Mh_r = m_halo_total * rh * rh / (rh + halo_a) ** 2 / c
    Mtot = Mh_r + m_disc_total * (1.0 - (1.0 + rh) * np.exp(-rh))
    sh = np.sqrt(np.maximum(Mtot, 0.0) / (3.0 * np.maximum(rh, 1e-12)))
    vh = sh[:, None] * g.standard_normal((n_halo, 3))
    pos = np.concatenate([xd, xh])
    vel = np.concatenate([vd, vh])
    mass = np.concatenate([np.full(n_disc, m_disc_total / max(n_disc, 1)),
                           np.full(n_halo, m_halo_total / max(n_halo, 1))])
    return pos.astype(dtype), vel.astype(dtype), mass.astype(dtype)


def clumps(n_per: int, centres, radius: float, seed: int, dtype=np.float64):
    """Compact Plummer clumps (scale ``radius``, truncated at 10 radius) of
    n_per particles each, centred at ``centres`` [k,3], masses 1/(k n_per):
    a multi-scale set whose clumps lie far apart relative to their size.
    The clumps are listed one after another (caller order)."""
    centres = np.asarray(centres, np.float64)
    parts = []
    for c, ctr in enumerate(centres):
        p, _ = plummer(n_per, seed + c)
        parts.append(ctr + radius * p)
    pos = np.concatenate(parts)
    m = np.full(len(pos), 1.0 / len(pos))
    return pos.astype(dtype), m.astype(dtype)


def target_sample(n: int, k: int, seed: int):
    """k distinct caller indices out of n, sorted (seeded)."""
    g = rng(seed)
    if k >= n:
        return np.arange(n, dtype=np.int64)
    return np.sort(g.choice(n, size=k, replace=False)).astype(np.int64)


# Named workloads (sizes and parameters of the evaluation configurations).
PLUMMER_16K = dict(kind="plummer", n=16384, seed=1000, dtype="f64", theta=0.7, eps=0.01)
DISC_1M = dict(kind="disc", n_disc=800_000, n_halo=200_000, seed=1001, dtype="f32",
               theta=0.5, eps=0.02, tau=1e-3, steps=10)
PLUMMER_10M = dict(kind="plummer", n=10_000_000, seed=1002, dtype="f32", thetas=(0.3, 0.5, 0.8),
                   eps=0.005, target_seed=2002)
PLUMMER_256K_GRAD = dict(kind="plummer", n=1 << 18, seed=1003, dtype="f32", theta=0.5, eps=0.01,
                         mass_seed=2003, fd_seed=3003, direct_n=4096, direct_seed=4003)
DISC_100M = dict(kind="disc", n_disc=20_000_000, n_halo=80_000_000, seed=1004, dtype="f32",
                 theta=0.5, eps=0.01, tau=1e-3)
