"""Pins of the g g -> t t~ (g g) Berends-Giele oracle.

1. g g -> t t~ against the closed form (Ellis, Stirling & Webber, QCD and
   Collider Physics, sec. 10; Combridge 1979):
     <|M|^2> = g^4 (1/(6 t1 t2) - 3/8)(t1^2 + t2^2 + rho - rho^2/(4 t1 t2)),
     t1 = 2 p1.p3/s, t2 = 2 p2.p3/s, rho = 4 m^2/s.
2. Parke-Taylor MHV amplitudes for a massless quark line and four gluons
   (Dixon, hep-ph/9601359): |A(qbar, q, g...)|^2 = s_{f-,j}^3 s_{f+,j} / (s_{qbar q}
   s_{q 1} ... s_{n qbar}) for exactly one negative-helicity gluon j (and the
   parity conjugate), zero for fewer; with t^a = T^a/sqrt(2) the oracle's
   partial amplitudes carry an extra g^(2n) 2^n.  This fixes the three- and
   four-gluon vertices including their normalisation.
3. Gauge invariance of every partial amplitude (eps_j -> k_j), Bose symmetry,
   Lorentz and azimuthal invariance, and the exact (alpha_s'/alpha_s)^4 ratio.
"""
import math

import numpy as np
import pytest

import synth
from oracle import qcd_bg
from oracle.lorentz import helicity_combinations, mdot

from kin import boost, rotate, rotation

RATIO = (0.130 / 0.118) ** 4


def _two_to_n(n_out, masses, root_s, seed):
    rng = np.random.default_rng(seed)
    n = 6
    fin = synth.rambo_massive(rng, n, masses, np.full(n, root_s)) if any(masses) else \
        synth.rambo_massless(rng, n, n_out, np.full(n, root_s))
    beams = np.zeros((n, 2, 4))
    beams[:, 0] = [root_s / 2, 0, 0, root_s / 2]
    beams[:, 1] = [root_s / 2, 0, 0, -root_s / 2]
    return np.concatenate([beams, fin], axis=1)


def test_gg_ttbar_closed_form():
    mt, gs = 173.0, 1.21
    for root_s in (400.0, 900.0, 3000.0):
        p = _two_to_n(2, [mt, mt], root_s, 11)
        s = root_s ** 2
        t1 = 2 * mdot(p[:, 0], p[:, 2]) / s
        t2 = 2 * mdot(p[:, 1], p[:, 2]) / s
        rho = 4 * mt * mt / s
        closed = gs ** 4 * (1 / (6 * t1 * t2) - 3 / 8) * (t1 ** 2 + t2 ** 2 + rho - rho ** 2 / (4 * t1 * t2))
        np.testing.assert_allclose(qcd_bg.me2_ttbar_gluons(p, gs, mt, 0), closed, rtol=1e-12)


def _mhv_check(p, gs):
    npart = p.shape[1]
    n = npart - 2
    inc, out = [0, 1], list(range(4, npart))
    slots = inc + out
    kout = p.copy()
    kout[:, :2] *= -1

    def s(a, b):
        return np.abs(2 * mdot(kout[:, a], kout[:, b]))

    worst, zero, count = 0.0, 0.0, 0
    for hel in helicity_combinations(npart):
        k, e, ub, v = qcd_bg.external_states(p, hel, 0.0, inc, out, 2, 3)
        amps = qcd_bg.partial_amplitudes(k, e, ub, v, p[:, 3], 0.0, gs)
        ho = list(hel)
        ho[0], ho[1] = -ho[0], -ho[1]                # crossing to all-outgoing helicities
        neg = [i for i in range(npart) if ho[i] < 0]
        pos = [i for i in range(npart) if ho[i] > 0]
        for pi, a in amps.items():
            got = np.abs(a) ** 2 / (gs ** (2 * n) * 2 ** n)
            if ho[2] == ho[3] or len(neg) <= 1 or len(pos) <= 1:
                zero = max(zero, float(np.max(got)))
                continue
            chain = [2] + [slots[x] for x in pi] + [3]
            den = s(3, 2)
            for x, y in zip(chain[:-1], chain[1:]):
                den = den * s(x, y)
            if len(neg) == 2:
                fm = 2 if ho[2] < 0 else 3
                j = [x for x in neg if x not in (2, 3)][0]
            elif len(pos) == 2:
                fm = 2 if ho[2] > 0 else 3
                j = [x for x in pos if x not in (2, 3)][0]
            else:
                continue                             # NMHV: no one-line formula
            fp = 5 - fm
            pred = s(fm, j) ** 3 * s(fp, j) / den
            worst = max(worst, float(np.max(np.abs(got / pred - 1))))
            count += 1
    return worst, zero, count


@pytest.mark.parametrize("n_out", [0, 2])
def test_parke_taylor_mhv(n_out):
    p = _two_to_n(n_out + 2, [0.0] * (n_out + 2), 900.0, 21)
    worst, zero, count = _mhv_check(p, 1.1)
    assert count > 0
    assert worst < 1e-10
    assert zero < 1e-25


def test_gauge_invariance_each_gluon():
    p = synth.events("gg_ttgg", 8)
    gs, mt = 1.2, 173.0
    inc, out = [0, 1], [4, 5]
    for hel in helicity_combinations(6)[::5]:
        k, e, ub, v = qcd_bg.external_states(p, hel, mt, inc, out, 2, 3)
        ref = qcd_bg.partial_amplitudes(k, e, ub, v, p[:, 3], mt, gs)
        scale = np.max(np.abs(np.stack(list(ref.values()))), axis=0)
        for slot in range(4):
            e2 = e.copy()
            e2[slot] = k[slot].astype(complex)
            amps = qcd_bg.partial_amplitudes(k, e2, ub, v, p[:, 3], mt, gs)
            for a in amps.values():
                assert np.all(np.abs(a) < 1e-11 * scale * np.abs(k[slot][:, 0]))


def test_bose_symmetry():
    p = synth.events("gg_ttgg", 6)
    base = qcd_bg.me2(p, synth.ORIG_QCD)
    sw = p.copy()
    sw[:, [4, 5]] = p[:, [5, 4]]
    np.testing.assert_allclose(qcd_bg.me2(sw, synth.ORIG_QCD), base, rtol=1e-11)
    sw = p.copy()
    sw[:, [0, 1]] = p[:, [1, 0]]
    np.testing.assert_allclose(qcd_bg.me2(sw, synth.ORIG_QCD), base, rtol=1e-11)


def test_lorentz_invariance():
    p = synth.events("gg_ttgg", 5)
    base = qcd_bg.me2(p, synth.ORIG_QCD)
    moved = boost(rotate(p, rotation([0.2, 1.0, -0.4], 0.9)), [0.1, 0.5, -0.3])
    np.testing.assert_allclose(qcd_bg.me2(moved, synth.ORIG_QCD), base, rtol=1e-10)


def test_alpha_s_ratio_exact():
    p = synth.events("gg_ttgg", 10)
    a = qcd_bg.me2(p, synth.ORIG_QCD)
    b = qcd_bg.me2(p, synth.NEW_QCD)
    np.testing.assert_allclose(b / a, RATIO, rtol=1e-13)
    assert math.isclose(RATIO, 1.47314460632146, rel_tol=1e-13)
