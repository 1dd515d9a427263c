"""Reweighting semantics of the oracle (paper, teaRex section): the
normaliser's 1/0 -> 0 guard and the normalise-then-multiply order."""
import numpy as np

import synth
from oracle import reweight


def test_zero_guard_and_order():
    m0 = np.array([2.0, 0.0, 4.0, 3.0])
    w = np.array([1.0, 5.0, -2.0, 0.0])
    norm = reweight.normalisation(w, m0)
    np.testing.assert_array_equal(norm, [0.5, 0.0, -0.5, 0.0])


def test_reweight_identity_card_gives_input_weights():
    p = synth.events("ee_mumu", 30)
    w = np.linspace(0.5, 2.0, 30)
    out, m0, mk = reweight.reweight("ee_mumu", p, w, synth.ORIG_EW, [synth.ORIG_EW, synth.NEW_EE])
    np.testing.assert_allclose(out[0], w, rtol=1e-15)
    np.testing.assert_array_equal(out[1], (w * (1.0 / m0)) * mk[1])


def test_zero_matrix_element_gives_zero_weight():
    # an event with all momenta zero except the beams has |M|^2 = nan; build a
    # true zero instead: alpha_s -> 0 makes u u~ -> e+e- g vanish identically
    import dataclasses
    p = synth.events("uu_eeg", 5)
    zero_card = dataclasses.replace(synth.ORIG_EW, aS=0.0)
    out, m0, _ = reweight.reweight("uu_eeg", p, np.ones(5), zero_card, [synth.NEW_UU])
    assert np.all(m0 == 0.0)
    np.testing.assert_array_equal(out, 0.0)
