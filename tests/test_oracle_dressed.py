"""Pins of the colour-dressed recursion (oracle/qcd_dressed.py), the oracle
of g g -> t t~ t t~.

1. Closed forms, spin- and colour-averaged, massless quarks unless stated
   (Ellis, Stirling & Webber, QCD and Collider Physics, table 7.1; Combridge
   1979 for heavy quarks):
     u u~ -> u u~ : g^4 [4/9 ((s^2 + u^2)/t^2 + (t^2 + u^2)/s^2) - 8/27 u^2/(s t)]
     u u  -> u u  : g^4 [4/9 ((s^2 + u^2)/t^2 + (s^2 + t^2)/u^2) - 8/27 s^2/(t u)]
     u u~ -> t t~ : g^4 4/9 ((m^2 - t)^2 + (m^2 - u)^2 + 2 m^2 s) / s^2
     g g  -> t t~ : the form of tests/test_oracle_gg.py.
   The first two fix the handling of identical quarks: the interference
   term's sign comes from the minus sign between the two pairings (the
   same-sign sum misses the closed form by 11%).
2. g g -> t t~ g against the colour-ordered recursion of oracle/qcd_bg.py (a
   different algorithm with its own pins); its four-gluon vertex enters here,
   and leaving it out breaks the agreement.
3. g g -> t t~ t t~: gauge invariance (either gluon's polarisation replaced
   by its momentum gives zero, per colour component, for each pairing alone
   and for their signed sum), Lorentz invariance, Bose symmetry of the
   gluons, symmetry under exchanging the two tops, exact alpha_s^4 scaling.
4. Helicity reversal, the relation the device kernels of the pure-QCD
   processes use to evaluate half of the helicities: with vector couplings,
   real coupling constants and real propagators, reversing every helicity
   conjugates each colour component of the amplitude up to one common phase,
   so the colour-summed |M_h|^2 is unchanged (massive tops included).
   Checked on g g -> t t~ g, g g -> t t~ g g and g g -> t t~ t t~ (both
   pairings) per helicity, to 1e-13 of the helicity sum; and the control
   that the relation does not hold with the chiral Z couplings and Z width of
   u u~ -> e+ e- g (oracle/uu_eeg.py), where the generator keeps every
   helicity.
"""

import numpy as np
import pytest

import synth
from oracle import qcd_bg, qcd_dressed as qd
from oracle.lorentz import mdot

from kin import boost

L = qd.Leg
GS, MT = 1.21, 173.0


def _two_to_two(masses, root_s, seed, n=5):
    rng = np.random.default_rng(seed)
    fin = synth.rambo_massive(rng, n, masses, np.full(n, root_s)) if any(masses) else \
        synth.rambo_massless(rng, n, 2, np.full(n, root_s))
    return _with_beams(fin, root_s)


def _with_beams(fin, root_s):
    n = fin.shape[0]
    beams = np.zeros((n, 2, 4))
    beams[:, 0] = [root_s / 2, 0, 0, root_s / 2]
    beams[:, 1] = [root_s / 2, 0, 0, -root_s / 2]
    return np.concatenate([beams, fin], axis=1)


def _mandelstam(p):
    s = mdot(p[:, 0] + p[:, 1], p[:, 0] + p[:, 1])
    t = mdot(p[:, 0] - p[:, 2], p[:, 0] - p[:, 2])
    u = mdot(p[:, 0] - p[:, 3], p[:, 0] - p[:, 3])
    return s, t, u


# u(0) u~(1) -> u(2) u~(3): the incoming quark and outgoing antiquark are column
# ends, the outgoing quark and incoming antiquark row ends.  Pairing 1 joins
# 0 -> 2 and 1 ... 3 (t channel), pairing 2 joins 1 ... 0 and 2 ... 3 (s channel).
UUBAR = [L("q", True), L("qb", True), L("q", False), L("qb", False)]
UUBAR_PAIRINGS = [(1.0, [(2, 0), (1, 3)]), (-1.0, [(2, 3), (1, 0)])]


def test_uubar_uubar_closed_form_and_exchange_sign():
    p = _two_to_two([0.0, 0.0], 900.0, 12)
    s, t, u = _mandelstam(p)
    closed = GS ** 4 * (4 / 9 * ((s ** 2 + u ** 2) / t ** 2 + (t ** 2 + u ** 2) / s ** 2) - 8 / 27 * u ** 2 / (s * t))
    got = qd.me2(p, UUBAR, UUBAR_PAIRINGS, GS, 0.25 / 9)
    np.testing.assert_allclose(got, closed, rtol=1e-12)
    same_sign = [(1.0, UUBAR_PAIRINGS[0][1]), (1.0, UUBAR_PAIRINGS[1][1])]
    assert np.max(np.abs(qd.me2(p, UUBAR, same_sign, GS, 0.25 / 9) / closed - 1.0)) > 0.01


def test_uu_uu_closed_form():
    legs = [L("q", True), L("q", True), L("q", False), L("q", False)]
    p = _two_to_two([0.0, 0.0], 700.0, 13)
    s, t, u = _mandelstam(p)
    closed = GS ** 4 * (4 / 9 * ((s ** 2 + u ** 2) / t ** 2 + (s ** 2 + t ** 2) / u ** 2) - 8 / 27 * s ** 2 / (t * u))
    got = qd.me2(p, legs, [(1.0, [(2, 0), (3, 1)]), (-1.0, [(3, 0), (2, 1)])], GS, 0.25 / 9)
    np.testing.assert_allclose(got, closed, rtol=1e-12)


def test_uubar_ttbar_closed_form():
    legs = [L("q", True), L("qb", True), L("q", False, MT), L("qb", False, MT)]
    for root_s in (400.0, 1500.0):
        p = _two_to_two([MT, MT], root_s, 14)
        s, t, u = _mandelstam(p)
        closed = GS ** 4 * 4 / 9 * ((MT ** 2 - t) ** 2 + (MT ** 2 - u) ** 2 + 2 * MT ** 2 * s) / s ** 2
        got = qd.me2(p, legs, [(1.0, [(2, 3), (1, 0)])], GS, 0.25 / 9)
        np.testing.assert_allclose(got, closed, rtol=1e-12)


def test_gg_ttbar_closed_form():
    legs = [L("g", True), L("g", True), L("q", False, MT), L("qb", False, MT)]
    for root_s in (400.0, 3000.0):
        p = _two_to_two([MT, MT], root_s, 11)
        s = root_s ** 2
        t1 = 2 * mdot(p[:, 0], p[:, 2]) / s
        t2 = 2 * mdot(p[:, 1], p[:, 2]) / s
        rho = 4 * MT * MT / s
        closed = GS ** 4 * (1 / (6 * t1 * t2) - 3 / 8) * (t1 ** 2 + t2 ** 2 + rho - rho ** 2 / (4 * t1 * t2))
        np.testing.assert_allclose(qd.me2(p, legs, [(1.0, [(2, 3)])], GS, 0.25 / 64), closed, rtol=1e-12)


def _ggttg_events():
    rng = np.random.default_rng(3)
    return _with_beams(synth.rambo_massive(rng, 3, [MT, MT, 0.0], np.full(3, 1500.0)), 1500.0)


GGTTG = [L("g", True), L("g", True), L("q", False, MT), L("qb", False, MT), L("g", False)]


def test_gg_ttbar_g_against_colour_ordered_recursion():
    p = _ggttg_events()
    np.testing.assert_allclose(qd.me2(p, GGTTG, [(1.0, [(2, 3)])], GS, 0.25 / 64),
                               qcd_bg.me2_ttbar_gluons(p, GS, MT, 1), rtol=1e-12)


def _no_v4(a, b, c, gs):
    """A four-gluon current of the right shape, zero."""
    legs = qd._merge(a.legs, b.legs, c.legs)
    dims = [a.arr.shape[0]]
    for leg in legs:
        src = next(x for x in (a, b, c) if leg in x.legs)
        dims.append(src.arr.shape[1 + src.legs.index(leg)])
    return qd.Current("g", legs, np.zeros(dims + [8, 4], dtype=complex), a.k + b.k + c.k)


def test_four_gluon_vertex_is_needed(monkeypatch):
    """A recursion without the four-gluon vertex misses the other oracle."""
    p = _ggttg_events()
    want = qcd_bg.me2_ttbar_gluons(p, GS, MT, 1)
    monkeypatch.setattr(qd, "v4_current", _no_v4)
    got = qd.me2(p, GGTTG, [(1.0, [(2, 3)])], GS, 0.25 / 64)
    assert np.max(np.abs(got / want - 1.0)) > 1e-3


def _tttt_events(n, seed):
    rng = np.random.default_rng(seed)
    return _with_beams(synth.rambo_massive(rng, n, [MT] * 4, np.full(n, 1500.0)), 1500.0)


@pytest.mark.parametrize("hel", [(1, -1, 1, 1, -1, 1), (-1, -1, 1, -1, 1, 1), (1, 1, -1, -1, -1, 1)])
def test_gg_tttt_gauge_invariance(hel):
    p = _tttt_events(2, 21)
    legs = qd.gg_tttt_legs(MT)
    amp = qd.amplitude_for(p, legs, qd.GG_TTTT_PAIRINGS, GS, hel)
    scale = np.abs(amp).reshape(2, -1).max(axis=1)
    assert np.all(scale > 0)
    for gauge in (0, 1):
        for pairings in (qd.GG_TTTT_PAIRINGS, qd.GG_TTTT_PAIRINGS[:1], qd.GG_TTTT_PAIRINGS[1:]):
            g = qd.amplitude_for(p, legs, pairings, GS, hel, gauge=gauge)
            assert np.all(np.abs(g).reshape(2, -1).max(axis=1) < 1e-12 * scale)


def test_gg_tttt_invariances_and_scaling():
    p = _tttt_events(1, 22)
    card = synth.ORIG_QCD
    m0 = qd.me2_gg_tttt(p, card)
    assert np.all(m0 > 0)
    np.testing.assert_allclose(qd.me2_gg_tttt(boost(p, [0.3, -0.2, 0.5]), card), m0, rtol=1e-12)
    np.testing.assert_allclose(qd.me2_gg_tttt(p[:, [1, 0, 2, 3, 4, 5]], card), m0, rtol=1e-12)
    np.testing.assert_allclose(qd.me2_gg_tttt(p[:, [0, 1, 4, 3, 2, 5]], card), m0, rtol=1e-12)
    new = synth.NEW_QCD
    np.testing.assert_allclose(qd.me2_gg_tttt(p, new) / m0, (new.aS / card.aS) ** 4, rtol=1e-12)


def _reversal_gap(p, legs, pairings, hels):
    """Largest | |M_h|^2 - |M_~h|^2 | over hels, per event, and the sum over
    hels of |M_h|^2 (colour-summed, per helicity)."""
    gap = np.zeros(p.shape[0])
    tot = np.zeros(p.shape[0])
    for hel in hels:
        a = qd.amplitude_for(p, legs, pairings, GS, hel)
        b = qd.amplitude_for(p, legs, pairings, GS, tuple(-h for h in hel))
        sa = np.sum(np.abs(a.reshape(p.shape[0], -1)) ** 2, axis=1)
        sb = np.sum(np.abs(b.reshape(p.shape[0], -1)) ** 2, axis=1)
        gap = np.maximum(gap, np.abs(sa - sb))
        tot += sa + sb
    return gap, tot


def test_reversed_helicities_equal_in_qcd():
    import itertools
    p = _ggttg_events()
    hels = [h for h in itertools.product((-1, 1), repeat=5) if h[0] == -1]
    gap, tot = _reversal_gap(p, GGTTG, [(1.0, [(2, 3)])], hels)
    assert np.all(tot > 0) and np.all(gap < 1e-13 * tot)
    rng = np.random.default_rng(31)
    p6 = _with_beams(synth.rambo_massive(rng, 2, [MT, MT, 0.0, 0.0], np.full(2, 1500.0)), 1500.0)
    gg_ttgg = GGTTG + [L("g", False)]
    hels6 = [(-1, 1, 1, -1, 1, 1), (-1, -1, 1, 1, -1, 1), (-1, 1, -1, -1, -1, -1), (-1, -1, -1, 1, 1, -1)]
    gap, tot = _reversal_gap(p6, gg_ttgg, [(1.0, [(2, 3)])], hels6)
    assert np.all(tot > 0) and np.all(gap < 1e-13 * tot)
    p4 = _tttt_events(2, 32)
    gap, tot = _reversal_gap(p4, qd.gg_tttt_legs(MT), qd.GG_TTTT_PAIRINGS, hels6)
    assert np.all(tot > 0) and np.all(gap < 1e-13 * tot)


def test_reversed_helicities_differ_with_z_exchange():
    import itertools
    from oracle import uu_eeg
    from oracle.couplings import Couplings
    p = synth.events("uu_eeg", 4, seed=33)
    c = Couplings.from_card(synth.ORIG_EW)
    hels = list(itertools.product((-1, 1), repeat=5))
    m = {h: np.abs(uu_eeg.amplitude(p, c, h)) ** 2 for h in hels}
    tot = sum(m.values())
    gap = np.max([np.abs(m[h] - m[tuple(-x for x in h)]) for h in hels], axis=0)
    assert np.all(gap > 0.05 * tot)
