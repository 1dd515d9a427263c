"""RAMBO phase-space generator (Kleiss, Stirling, Ellis, Comput. Phys. Commun.
40 (1986) 359), vectorised over events with NumPy.

This module only produces input momenta.  It holds none of the matrix-element
arithmetic and is shared by the oracle-side tests and the device-side tests
and benchmark alike.

Momenta are (E, px, py, pz) in GeV, in the centre-of-mass frame of the
incoming pair.
"""
from __future__ import annotations

import math

import numpy as np


def rambo_massless(rng: np.random.Generator, n_events: int, n_out: int,
                   sqrt_s: np.ndarray) -> np.ndarray:
    """n_out massless momenta per event with total momentum (sqrt_s, 0, 0, 0).

    Steps of the published algorithm: draw n_out isotropic massless vectors
    with energy density q0*exp(-q0), then boost and rescale their sum to the
    requested total momentum.  Returns an array of shape [n_events, n_out, 4].
    """
    sqrt_s = np.broadcast_to(np.asarray(sqrt_s, dtype=np.float64), (n_events,))
    r = rng.random((n_events, n_out, 4))
    cos_t = 2.0 * r[..., 0] - 1.0
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    phi = 2.0 * math.pi * r[..., 1]
    # -log(r1*r2) has density q0*exp(-q0); 1-r keeps the argument in (0, 1].
    q0 = -np.log((1.0 - r[..., 2]) * (1.0 - r[..., 3]))
    q = np.empty((n_events, n_out, 4))
    q[..., 0] = q0
    q[..., 1] = q0 * sin_t * np.cos(phi)
    q[..., 2] = q0 * sin_t * np.sin(phi)
    q[..., 3] = q0 * cos_t

    big_q = q.sum(axis=1)                                   # [n, 4]
    mass = np.sqrt(big_q[:, 0] ** 2 - np.sum(big_q[:, 1:] ** 2, axis=1))
    b = -big_q[:, 1:] / mass[:, None]                        # [n, 3]
    x = sqrt_s / mass
    gamma = big_q[:, 0] / mass
    a = 1.0 / (1.0 + gamma)

    bq = np.einsum("nj,nij->ni", b, q[..., 1:])              # b . q_i
    p = np.empty_like(q)
    p[..., 0] = x[:, None] * (gamma[:, None] * q[..., 0] + bq)
    p[..., 1:] = x[:, None, None] * (
        q[..., 1:] + b[:, None, :] * q[..., 0:1] + (a[:, None] * bq)[..., None] * b[:, None, :])
    return p


def massless_weight(n_out: int, s: float) -> float:
    """Phase-space volume of n_out massless particles for the measure
    prod_i d^3p_i / (2 E_i) delta^4(P - sum p_i), no factors of 2*pi.

    RAMBO produces every massless configuration with this same constant
    weight (the closed form is in the cited paper)."""
    n = n_out
    return (math.pi / 2.0) ** (n - 1) * s ** (n - 2) / (math.factorial(n - 1) * math.factorial(n - 2))


def rambo_massive(rng: np.random.Generator, n_events: int, masses, sqrt_s: np.ndarray,
                  newton_iters: int = 60) -> np.ndarray:
    """Massive momenta by rescaling a massless RAMBO point (same paper):
    solve sum_i sqrt(m_i^2 + xi^2 E_i^2) = sqrt_s for xi by Newton's method,
    then k_i = (sqrt(m_i^2 + xi^2 E_i^2), xi * p_i)."""
    masses = np.asarray(masses, dtype=np.float64)
    n_out = masses.size
    sqrt_s = np.broadcast_to(np.asarray(sqrt_s, dtype=np.float64), (n_events,))
    p = rambo_massless(rng, n_events, n_out, sqrt_s)
    e = p[..., 0]
    m2 = masses[None, :] ** 2
    xi = np.sqrt(np.maximum(0.0, 1.0 - (masses.sum() / sqrt_s) ** 2))
    for _ in range(newton_iters):
        ek = np.sqrt(m2 + (xi[:, None] * e) ** 2)
        f = ek.sum(axis=1) - sqrt_s
        df = (xi[:, None] * e * e / ek).sum(axis=1)
        step = f / df
        xi = xi - step
        if np.max(np.abs(step / xi)) < 1e-16:
            break
    k = np.empty_like(p)
    k[..., 0] = np.sqrt(m2 + (xi[:, None] * e) ** 2)
    k[..., 1:] = xi[:, None, None] * p[..., 1:]
    return k
