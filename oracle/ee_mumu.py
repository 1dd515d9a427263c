"""e+(p0) e-(p1) -> mu+(p2) mu-(p3) through s-channel photon and Z, FP64.

Two Feynman diagrams, written out with explicit 4x4 Dirac matrices:

  M = sum_{V = gamma, Z} [vbar(p0) G_V^mu u(p1)] D^V_{mu nu}(q) [ubar(p3) G_V^nu v(p2)]

with G_V^mu = -i gamma^mu (cL P_L + cR P_R) (``couplings``), q = p0 + p1,
D^gamma = -i g_{mu nu}/q^2 and the fixed-width unitary-gauge Z propagator
D^Z = -i (g_{mu nu} - q_mu q_nu / M_Z^2) / (q^2 - M_Z^2 + i M_Z Gamma_Z).
|M|^2 is summed over all 16 helicities and multiplied by the spin average 1/4.

Pinned by the textbook helicity-amplitude closed form for massless fermions
(tests/test_oracle_ee.py).
"""
from __future__ import annotations

import numpy as np

from .couplings import Couplings
from .lorentz import GAMMA, PL, PR, bar, helicity_combinations, mdot, u_spinor, v_spinor

SPIN_AVERAGE = 0.25


def vertex(cl, cr):
    """-i gamma^mu (cL P_L + cR P_R), shape [4 (mu), 4, 4]."""
    return -1j * np.einsum("mij,jk->mik", GAMMA, cl * PL + cr * PR)


def current(row, gam, col):
    """row . Gamma^mu . col for row/col spinors [N, 4]; returns j^mu [N, 4]."""
    return np.einsum("ni,mij,nj->nm", row, gam, col)


def propagate(j1, j2, q, mass, width):
    """j1^mu D_{mu nu}(q) j2^nu for a photon (mass = 0) or the Z."""
    q2 = mdot(q, q)
    if mass == 0.0:
        return -1j * mdot(j1, j2) / q2
    num = mdot(j1, j2) - mdot(q, j1) * mdot(q, j2) / mass ** 2
    return -1j * num / (q2 - mass ** 2 + 1j * mass * width)


def me2(p: np.ndarray, card) -> np.ndarray:
    """Spin-averaged |M|^2 per event; p has shape [N, 4, 4]."""
    c = Couplings.from_card(card)
    q = p[:, 0] + p[:, 1]
    bosons = [(c.photon("e"), c.photon("mu"), 0.0, 0.0),
              (c.zboson("e"), c.zboson("mu"), c.mz, c.wz)]
    total = np.zeros(p.shape[0])
    for h0, h1, h2, h3 in helicity_combinations(4):
        vb = bar(v_spinor(p[:, 0], 0.0, h0))
        u = u_spinor(p[:, 1], 0.0, h1)
        v = v_spinor(p[:, 2], 0.0, h2)
        ub = bar(u_spinor(p[:, 3], 0.0, h3))
        amp = np.zeros(p.shape[0], dtype=complex)
        for (ce, cm, mass, width) in bosons:
            je = current(vb, vertex(*ce), u)
            jm = current(ub, vertex(*cm), v)
            amp += propagate(je, jm, q, mass, width)
        total += np.abs(amp) ** 2
    return SPIN_AVERAGE * total

