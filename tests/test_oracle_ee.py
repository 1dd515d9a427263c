"""Pin of the e+e- -> mu+mu- oracle against the textbook closed form.

For massless fermions and theta the angle between e- and mu- (e.g. Peskin &
Schroeder sec. 5.2 with chiral Z couplings):

  <|M|^2> = e^4/4 sum_{i, j in L, R} |A_ij|^2 (1 + s_ij cos(theta))^2,
  s_ij = +1 for i = j, -1 otherwise,
  A_ij = Q_e Q_mu + g_i g_j /(s_W^2 c_W^2) * s/(s - M_Z^2 + i M_Z Gamma_Z),
  g_L = -1/2 + s_W^2, g_R = s_W^2.

The oracle sums Feynman diagrams with 4x4 Dirac matrices, so this is an
independent closed form, not the oracle's own formula.
"""
import math

import numpy as np

import synth
from oracle import ee_mumu, reweight


def closed_form(cos_t, card, sqrt_s=200.0):
    s = sqrt_s ** 2
    e2 = 4 * math.pi / card.aEWM1
    sw2 = card.sw2
    g = {"L": -0.5 + sw2, "R": sw2}
    prop = s / (s - card.MZ ** 2 + 1j * card.MZ * card.WZ)
    total = 0.0
    for i in "LR":
        for j in "LR":
            a = 1.0 + g[i] * g[j] / (sw2 * (1 - sw2)) * prop
            sign = 1.0 if i == j else -1.0
            total = total + abs(a) ** 2 * (1 + sign * cos_t) ** 2
    return e2 ** 2 / 4 * total


def test_closed_form_original_and_new_card():
    p = synth.events("ee_mumu", 400)
    cos_t = p[:, 2, 3] / p[:, 2, 0]          # mu+ along n  =>  angle(e-, mu-) = theta
    for card in (synth.ORIG_EW, synth.NEW_EE):
        np.testing.assert_allclose(ee_mumu.me2(p, card), closed_form(cos_t, card), rtol=1e-13)


def test_closed_form_at_fixed_angles():
    cos_t = np.array([-1.0, -0.5, 0.0, 0.5, 1.0])
    sin_t = np.sqrt(1 - cos_t ** 2)
    p = np.zeros((5, 4, 4))
    p[:, 0] = [100, 0, 0, 100]
    p[:, 1] = [100, 0, 0, -100]
    p[:, 2, 0] = 100
    p[:, 2, 1] = 100 * sin_t
    p[:, 2, 3] = 100 * cos_t
    p[:, 3] = p[:, 0] + p[:, 1] - p[:, 2]
    for card in (synth.ORIG_EW, synth.NEW_EE):
        np.testing.assert_allclose(ee_mumu.me2(p, card), closed_form(cos_t, card), rtol=1e-13)
    w, m0, mk = reweight.reweight("ee_mumu", p, np.ones(5), synth.ORIG_EW, [synth.NEW_EE])
    np.testing.assert_allclose(w[0], closed_form(cos_t, synth.NEW_EE) / closed_form(cos_t, synth.ORIG_EW),
                               rtol=1e-13)
