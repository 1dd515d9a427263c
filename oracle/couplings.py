"""Couplings from a parameter card (FP64).

Inputs are independent: 1/alpha, sin^2(theta_W), M_Z, Gamma_Z, alpha_s, m_t.
Vertex rules (textbook electroweak and QCD Feynman rules):

* photon - fermion f:  -i e Q_f gamma^mu
* Z - fermion f:       -i e/(s_W c_W) gamma^mu (gL P_L + gR P_R),
                        gL = T3_f - Q_f s_W^2, gR = -Q_f s_W^2
* gluon - quark:        i g_s gamma^mu t^a,  t^a = lambda^a / 2
* e = sqrt(4 pi / (1/alpha)), g_s = sqrt(4 pi alpha_s).
"""
from __future__ import annotations

import dataclasses
import math

# (charge Q, weak isospin T3) of the fermions the processes use.
FERMIONS = {
    "e": (-1.0, -0.5),
    "mu": (-1.0, -0.5),
    "u": (2.0 / 3.0, 0.5),
}


@dataclasses.dataclass(frozen=True)
class Couplings:
    e: float
    sw: float
    cw: float
    gs: float
    mz: float
    wz: float
    mt: float

    @staticmethod
    def from_card(card) -> "Couplings":
        e = math.sqrt(4.0 * math.pi / card.aEWM1)
        sw = math.sqrt(card.sw2)
        cw = math.sqrt(1.0 - card.sw2)
        return Couplings(e=e, sw=sw, cw=cw, gs=math.sqrt(4.0 * math.pi * card.aS),
                         mz=card.MZ, wz=card.WZ, mt=card.MT)

    def photon(self, f):
        """(cL, cR) of the photon vertex -i gamma^mu (cL P_L + cR P_R)."""
        q, _ = FERMIONS[f]
        return self.e * q, self.e * q

    def zboson(self, f):
        """(cL, cR) of the Z vertex -i gamma^mu (cL P_L + cR P_R)."""
        q, t3 = FERMIONS[f]
        k = self.e / (self.sw * self.cw)
        return k * (t3 - q * self.sw ** 2), k * (-q * self.sw ** 2)
