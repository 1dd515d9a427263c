"""u(p0) u~(p1) -> e+(p2) e-(p3) g(p4) through photon and Z, FP64.

Four Feynman diagrams (boson gamma or Z, gluon emitted from the u or the u~
leg), written out with explicit 4x4 Dirac matrices:

  H_V^mu = vbar(p1) [ G_V^mu S(p0 - p4) E + E S(p0 - q) G_V^mu ] u(p0)
  M      = sum_V H_V^mu D^V_{mu nu}(q) [ubar(p3) G_V^nu v(p2)]

where q = p2 + p3, E = i g_s eps*(p4)-slash (the gluon vertex without its
colour matrix), S(k) = i k-slash / k^2 (massless quark propagator) and G_V, D^V
as in ``ee_mumu``.  Both diagrams carry the colour factor t^a_{ji}, whose sum
over colours is Tr(t^a t^a) = 4.  |M|^2 is summed over all 32 helicities and
averaged over spins (1/4) and colours (1/9).

Pinned by: the lepton-angle average against the textbook q q~ -> V* g closed
form, gauge invariance (eps -> k gives 0), Lorentz and phase invariance, and
exact linear scaling with alpha_s (tests/test_oracle_uu.py).
"""
from __future__ import annotations

import numpy as np

from .couplings import Couplings
from .ee_mumu import current, propagate, vertex
from .lorentz import bar, helicity_combinations, polarisation, slash, u_spinor, v_spinor

SPIN_COLOUR_AVERAGE = 0.25 / 9.0
COLOUR_SUM = 4.0      # sum over a, i, j of |t^a_ji|^2


def quark_propagator(k):
    """i k-slash / k^2 for a massless quark, shape [N, 4, 4]."""
    k2 = k[:, 0] ** 2 - k[:, 1] ** 2 - k[:, 2] ** 2 - k[:, 3] ** 2
    return 1j * slash(k) / k2[:, None, None]


def amplitude(p, c: Couplings, hel, gluon_pol=None):
    """Colour-stripped amplitude for one helicity assignment (h0..h4).

    ``gluon_pol`` replaces eps*(p4) (used by the gauge-invariance pin)."""
    h0, h1, h2, h3, h4 = hel
    u = u_spinor(p[:, 0], 0.0, h0)
    vb = bar(v_spinor(p[:, 1], 0.0, h1))
    v = v_spinor(p[:, 2], 0.0, h2)
    ub = bar(u_spinor(p[:, 3], 0.0, h3))
    eps = np.conj(polarisation(p[:, 4], h4)) if gluon_pol is None else gluon_pol
    emit = 1j * c.gs * slash(eps)                       # [N, 4, 4]
    q = p[:, 2] + p[:, 3]
    s_u = quark_propagator(p[:, 0] - p[:, 4])           # after emission off u
    s_ub = quark_propagator(p[:, 0] - q)                # before emission off u~
    amp = np.zeros(p.shape[0], dtype=complex)
    for cq, cl, mass, width in [(c.photon("u"), c.photon("e"), 0.0, 0.0),
                                (c.zboson("u"), c.zboson("e"), c.mz, c.wz)]:
        g_q = vertex(*cq)                               # [4, 4, 4]
        first = np.einsum("mij,njk,nkl->nmil", g_q, s_u, emit)
        second = np.einsum("nij,njk,mkl->nmil", emit, s_ub, g_q)
        h = np.einsum("ni,nmij,nj->nm", vb, first + second, u)
        lep = current(ub, vertex(*cl), v)
        amp += propagate(h, lep, q, mass, width)
    return amp


def me2(p: np.ndarray, card) -> np.ndarray:
    """Spin- and colour-averaged |M|^2 per event; p has shape [N, 5, 4]."""
    c = Couplings.from_card(card)
    total = np.zeros(p.shape[0])
    for hel in helicity_combinations(5):
        total += np.abs(amplitude(p, c, hel)) ** 2
    return SPIN_COLOUR_AVERAGE * COLOUR_SUM * total
