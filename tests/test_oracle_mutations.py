"""Planted mistakes in the oracle (on the CPU) must each fail one of the pins.

Each case patches one plausible error into the oracle - a dropped term, a
wrong sign, a wrong spinor type, a swapped coupling - and checks that the
corresponding pin from the other oracle tests detects it.
"""
import numpy as np

import synth
from oracle import ee_mumu, lorentz, qcd_bg, uu_eeg
from oracle.couplings import Couplings

import test_oracle_ee as tee
import test_oracle_gg as tgg
import test_oracle_uu as tuu


def _ee_error():
    p = synth.events("ee_mumu", 50)
    cos_t = p[:, 2, 3] / p[:, 2, 0]
    return np.max(np.abs(ee_mumu.me2(p, synth.ORIG_EW) / tee.closed_form(cos_t, synth.ORIG_EW) - 1))


def _ggtt_error():
    p = tgg._two_to_n(2, [173.0, 173.0], 900.0, 3)
    s = 900.0 ** 2
    t1 = 2 * lorentz.mdot(p[:, 0], p[:, 2]) / s
    t2 = 2 * lorentz.mdot(p[:, 1], p[:, 2]) / s
    rho = 4 * 173.0 ** 2 / s
    closed = 1.2 ** 4 * (1 / (6 * t1 * t2) - 3 / 8) * (t1 ** 2 + t2 ** 2 + rho - rho ** 2 / (4 * t1 * t2))
    return np.max(np.abs(qcd_bg.me2_ttbar_gluons(p, 1.2, 173.0, 0) / closed - 1))


def _uu_error():
    p = synth.events("uu_eeg", 10)
    six = tuu._lepton_octahedron(p)
    avg = np.mean([uu_eeg.me2(ev, synth.ORIG_EW) for ev in six], axis=0)
    return np.max(np.abs(avg / tuu._closed_form_average(p, synth.ORIG_EW) - 1))


def test_unpatched_baselines_pass():
    assert _ee_error() < 1e-12
    assert _ggtt_error() < 1e-12
    assert _uu_error() < 1e-11


def test_wrong_z_coupling_sign(monkeypatch):
    orig = Couplings.zboson

    def bad(self, f):
        cl, cr = orig(self, f)
        return cl, -cr
    monkeypatch.setattr(Couplings, "zboson", bad)
    assert _ee_error() > 1e-4
    assert _uu_error() > 1e-4


def test_width_without_mass_factor(monkeypatch):
    # (q^2 - M^2 + i Gamma) instead of (q^2 - M^2 + i M Gamma); a flipped width
    # sign would not be a mistake: with real couplings |M|^2 does not depend on it
    from oracle.lorentz import mdot

    def bad(j1, j2, q, mass, width):
        q2 = mdot(q, q)
        if mass == 0.0:
            return -1j * mdot(j1, j2) / q2
        num = mdot(j1, j2) - mdot(q, j1) * mdot(q, j2) / mass ** 2
        return -1j * num / (q2 - mass ** 2 + 1j * width)
    monkeypatch.setattr(ee_mumu, "propagate", bad)
    monkeypatch.setattr(uu_eeg, "propagate", bad)
    assert _ee_error() > 1e-4
    assert _uu_error() > 1e-4


def test_three_gluon_vertex_sign(monkeypatch):
    orig = qcd_bg.v3
    monkeypatch.setattr(qcd_bg, "v3", lambda *a: -orig(*a))
    assert _ggtt_error() > 1e-3


def test_dropped_four_gluon_vertex(monkeypatch):
    monkeypatch.setattr(qcd_bg, "v4", lambda ja, jb, jc: 0 * ja)
    p = tgg._two_to_n(4, [0.0] * 4, 900.0, 21)
    worst, _, _ = tgg._mhv_check(p, 1.1)
    assert worst > 1e-3


def test_antitop_with_u_spinor(monkeypatch):
    monkeypatch.setattr(qcd_bg, "v_spinor", lorentz.u_spinor)
    assert _ggtt_error() > 1e-3


def test_massive_propagator_sign(monkeypatch):
    # replace (q-slash + m) by (q-slash - m) in the top propagator
    orig_eye = np.eye

    class FakeNp:
        def __getattr__(self, name):
            return getattr(np, name)

        @staticmethod
        def eye(n, *a, **k):
            return -orig_eye(n, *a, **k)
    monkeypatch.setattr(qcd_bg, "np", FakeNp())
    assert _ggtt_error() > 1e-3


def test_uu_dropped_diagram(monkeypatch):
    orig = uu_eeg.quark_propagator
    calls = {"n": 0}

    def bad(k):
        calls["n"] += 1
        out = orig(k)
        return out if calls["n"] % 2 else 0 * out
    monkeypatch.setattr(uu_eeg, "quark_propagator", bad)
    assert _uu_error() > 1e-3
