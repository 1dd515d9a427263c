"""Pins of the u u~ -> e+e- g oracle.

1. Lepton-angle average against the textbook q q~ -> V* g closed form.  With
   the lepton pair direction averaged in the V* rest frame (exact with the six
   octahedron directions, since |M|^2 is quadratic in the lepton direction),
   the lepton tensor becomes 4/3 (q^mu q^nu - Q^2 g^{mu nu}) and

     <|M|^2> = 1/36 * (1/4) sum_{ij} |A_ij|^2 * 4 e^4/(3 Q^2)
               * 32 g_s^2 (t^2 + u^2 + 2 s Q^2)/(t u)

   where 32 e_q^2 e^2 g_s^2 (t^2 + u^2 + 2 s Q^2)/(t u) is the spin- and
   colour-summed q q~ -> gamma* g result (its Q^2 -> 0 limit is the textbook
   8/9 (t/u + u/t) of q q~ -> g gamma after the 1/36 average), and
   A_ij = Q_u Q_e + g^u_i g^e_j/(s_W^2 c_W^2) Q^2/(Q^2 - M_Z^2 + i M_Z Gamma_Z)
   replaces Q_u Q_e for quark chirality i and lepton chirality j.
2. Gauge invariance: eps*(g) -> k(g) gives a vanishing amplitude.
3. Lorentz invariance, azimuthal-rotation invariance, exact linear alpha_s
   scaling.
"""
import dataclasses
import math

import numpy as np

import synth
from oracle import uu_eeg
from oracle.couplings import Couplings
from oracle.lorentz import helicity_combinations, polarisation

from kin import boost, boost_from_rest, mdot, rotate, rotation


def _closed_form_average(p, card):
    c = Couplings.from_card(card)
    q = p[:, 2] + p[:, 3]
    q2 = mdot(q, q)
    s = mdot(p[:, 0] + p[:, 1], p[:, 0] + p[:, 1])
    t = mdot(p[:, 0] - p[:, 4], p[:, 0] - p[:, 4])
    u = mdot(p[:, 1] - p[:, 4], p[:, 1] - p[:, 4])
    sw2 = card.sw2
    gu = {"L": 0.5 - 2 / 3 * sw2, "R": -2 / 3 * sw2}
    ge = {"L": -0.5 + sw2, "R": sw2}
    prop = q2 / (q2 - card.MZ ** 2 + 1j * card.MZ * card.WZ)
    amp2 = sum(abs(-2 / 3 + gu[i] * ge[j] / (sw2 * (1 - sw2)) * prop) ** 2 for i in "LR" for j in "LR")
    return (1 / 36) * (amp2 / 4) * (4 * c.e ** 4 / (3 * q2)) * 32 * c.gs ** 2 * (t * t + u * u + 2 * s * q2) / (t * u)


def _lepton_octahedron(p):
    """Six copies of each event with the lepton pair along +-x, +-y, +-z in the
    V* rest frame (same V* momentum); returns [6, N, 5, 4]."""
    q = p[:, 2] + p[:, 3]
    mq = np.sqrt(mdot(q, q))
    out = []
    for axis in range(3):
        for sign in (1.0, -1.0):
            lm = np.zeros((p.shape[0], 4))
            lm[:, 0] = mq / 2
            lm[:, 1 + axis] = sign * mq / 2
            lp = lm.copy()
            lp[:, 1:] *= -1
            ev = p.copy()
            ev[:, 2] = boost_from_rest(lp, q)
            ev[:, 3] = boost_from_rest(lm, q)
            out.append(ev)
    return np.stack(out)


def test_lepton_average_closed_form():
    p = synth.events("uu_eeg", 60)
    six = _lepton_octahedron(p)
    for card in (synth.ORIG_EW, synth.NEW_UU):
        avg = np.mean([uu_eeg.me2(ev, card) for ev in six], axis=0)
        np.testing.assert_allclose(avg, _closed_form_average(p, card), rtol=1e-12)


def test_octahedron_average_is_exact():
    # a different rotation of the six directions gives the same average
    p = synth.events("uu_eeg", 20)
    six = _lepton_octahedron(p)
    a = np.mean([uu_eeg.me2(ev, synth.ORIG_EW) for ev in six], axis=0)
    r = rotation([0.3, -0.5, 0.8], 0.7)
    q = p[:, 2] + p[:, 3]
    rot = []
    for ev in six:
        # rotate the lepton pair inside the V* rest frame
        beta = q / q[:, :1]
        lm_rest = np.stack([boost(ev[i, 3], -beta[i, 1:]) for i in range(len(ev))])
        lm_rest = rotate(lm_rest, r)
        lp_rest = lm_rest.copy()
        lp_rest[:, 1:] *= -1
        e2 = ev.copy()
        e2[:, 3] = boost_from_rest(lm_rest, q)
        e2[:, 2] = boost_from_rest(lp_rest, q)
        rot.append(uu_eeg.me2(e2, synth.ORIG_EW))
    np.testing.assert_allclose(np.mean(rot, axis=0), a, rtol=1e-12)


def test_gauge_invariance():
    p = synth.events("uu_eeg", 50)
    c = Couplings.from_card(synth.ORIG_EW)
    k = p[:, 4].astype(complex)
    for hel in helicity_combinations(5):
        ref = uu_eeg.amplitude(p, c, hel)
        eps = np.conj(polarisation(p[:, 4], hel[4]))
        ref_scale = np.abs(uu_eeg.amplitude(p, c, hel[:4] + (1,))) + np.abs(uu_eeg.amplitude(p, c, hel[:4] + (-1,)))
        gauge = uu_eeg.amplitude(p, c, hel, gluon_pol=k)
        assert np.all(np.abs(gauge) <= 1e-12 * (ref_scale + 1e-300) * p[:, 4, 0])
        assert eps.shape == k.shape and ref.shape == gauge.shape


def test_lorentz_and_rotation_invariance():
    p = synth.events("uu_eeg", 80)
    base = uu_eeg.me2(p, synth.ORIG_EW)
    moved = boost(rotate(p, rotation([1, 2, 3], 1.1)), [0.3, -0.4, 0.5])
    np.testing.assert_allclose(uu_eeg.me2(moved, synth.ORIG_EW), base, rtol=1e-11)
    azim = rotate(p, rotation([0, 0, 1], 2.3))
    np.testing.assert_allclose(uu_eeg.me2(azim, synth.ORIG_EW), base, rtol=1e-12)


def test_alpha_s_linear():
    p = synth.events("uu_eeg", 40)
    a = uu_eeg.me2(p, synth.ORIG_EW)
    b = uu_eeg.me2(p, dataclasses.replace(synth.ORIG_EW, aS=0.3))
    np.testing.assert_allclose(b / a, 0.3 / 0.118, rtol=1e-14)
    assert math.isfinite(float(a.sum()))
