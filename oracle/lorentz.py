"""Dirac matrices and external wavefunctions, FP64, vectorised over events.

Conventions (textbook; e.g. Peskin & Schroeder ch. 3 and the HELAS manual,
KEK-91-11, for the helicity basis):

* metric diag(+1, -1, -1, -1); four-vectors (E, px, py, pz), upper index;
* chiral (Weyl) representation, gamma^0 = [[0, 1], [1, 0]],
  gamma^i = [[0, s_i], [-s_i, 0]], gamma^5 = diag(-1, -1, +1, +1);
* helicity 2-spinors chi_+(n) = (cos(t/2), e^{i f} sin(t/2)),
  chi_-(n) = (-e^{-i f} sin(t/2), cos(t/2)) for n = (t, f);
* u(p, l) = (sqrt(E - l|p|) chi_l, sqrt(E + l|p|) chi_l),
  v(p, l) = (sqrt(E + l|p|) chi_-l, -sqrt(E - l|p|) chi_-l),
  ubar = u^dagger gamma^0, vbar = v^dagger gamma^0;
* eps(k, l) = (-l e1 - i e2)/sqrt(2), e1 = (0, cos t cos f, cos t sin f, -sin t),
  e2 = (0, -sin f, cos f, 0); an outgoing vector boson takes eps*.

Pinned by tests: Dirac equation, spinor completeness and normalisation,
helicity eigenvalues, transversality and orthonormality of eps.
"""
from __future__ import annotations

import numpy as np

I2 = np.eye(2, dtype=complex)
SIGMA = np.array([
    [[1, 0], [0, 1]],
    [[0, 1], [1, 0]],
    [[0, -1j], [1j, 0]],
    [[1, 0], [0, -1]],
], dtype=complex)

GAMMA = np.zeros((4, 4, 4), dtype=complex)
GAMMA[0] = np.block([[np.zeros((2, 2)), I2], [I2, np.zeros((2, 2))]])
for _i in range(1, 4):
    GAMMA[_i] = np.block([[np.zeros((2, 2)), SIGMA[_i]], [-SIGMA[_i], np.zeros((2, 2))]])
GAMMA5 = np.diag([-1.0, -1.0, 1.0, 1.0]).astype(complex)
PL = 0.5 * (np.eye(4) - GAMMA5)
PR = 0.5 * (np.eye(4) + GAMMA5)
METRIC = np.diag([1.0, -1.0, -1.0, -1.0])


def mdot(a, b):
    """Minkowski product a.b over the last axis (no complex conjugation)."""
    return a[..., 0] * b[..., 0] - a[..., 1] * b[..., 1] - a[..., 2] * b[..., 2] - a[..., 3] * b[..., 3]


def slash(a):
    """a_mu gamma^mu, shape [..., 4, 4]."""
    return (a[..., 0, None, None] * GAMMA[0] - a[..., 1, None, None] * GAMMA[1]
            - a[..., 2, None, None] * GAMMA[2] - a[..., 3, None, None] * GAMMA[3])


def _angles(p):
    pabs = np.sqrt(p[..., 1] ** 2 + p[..., 2] ** 2 + p[..., 3] ** 2)
    theta = np.arccos(np.clip(p[..., 3] / pabs, -1.0, 1.0))
    phi = np.arctan2(p[..., 2], p[..., 1])
    return pabs, theta, phi


def chi(p, lam):
    """Helicity eigen 2-spinor along the direction of p, helicity lam/2."""
    _, theta, phi = _angles(p)
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    out = np.empty(p.shape[:-1] + (2,), dtype=complex)
    if lam > 0:
        out[..., 0] = c
        out[..., 1] = np.exp(1j * phi) * s
    else:
        out[..., 0] = -np.exp(-1j * phi) * s
        out[..., 1] = c
    return out


def _roots(p, m, lam):
    """(sqrt(E - lam|p|), sqrt(E + lam|p|)); the smaller one as m/sqrt(E+|p|) so
    that it is exactly 0 for m = 0."""
    pabs = np.sqrt(p[..., 1] ** 2 + p[..., 2] ** 2 + p[..., 3] ** 2)
    big = np.sqrt(p[..., 0] + pabs)
    small = m / big
    return (small, big) if lam > 0 else (big, small)


def u_spinor(p, m, lam):
    minus, plus = _roots(p, m, lam)
    x = chi(p, lam)
    return np.concatenate([minus[..., None] * x, plus[..., None] * x], axis=-1)


def v_spinor(p, m, lam):
    minus, plus = _roots(p, m, lam)     # sqrt(E - lam|p|), sqrt(E + lam|p|)
    x = chi(p, -lam)
    return np.concatenate([plus[..., None] * x, -minus[..., None] * x], axis=-1)


def bar(psi):
    """Dirac adjoint psi^dagger gamma^0 as a row spinor."""
    return np.einsum("...i,ij->...j", np.conj(psi), GAMMA[0])


def polarisation(k, lam):
    """eps^mu(k, lam) for a massless vector boson of helicity lam = +-1."""
    _, theta, phi = _angles(k)
    ct, st, cf, sf = np.cos(theta), np.sin(theta), np.cos(phi), np.sin(phi)
    zero = np.zeros_like(ct)
    e1 = np.stack([zero, ct * cf, ct * sf, -st], axis=-1)
    e2 = np.stack([zero, -sf, cf, zero], axis=-1)
    return (-lam * e1 - 1j * e2) / np.sqrt(2.0)


def helicity_combinations(n):
    """All 2^n helicity assignments, each entry +-1."""
    grid = np.array(np.meshgrid(*[[-1, 1]] * n, indexing="ij")).reshape(n, -1).T
    return [tuple(int(x) for x in row) for row in grid]
