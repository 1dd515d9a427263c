"""Hand-computed pins of the reweighted cross section and its error."""
import math

import numpy as np

from oracle import xsec


def test_hand_computed_case():
    w = [1.0, 2.0, 3.0]
    wp = [2.0, 4.0, 6.0]
    xs, err, bad = xsec.xsec(w, wp, sigma=10.0, dsigma=0.5, norm=0.25)
    # sigma' = 0.25 * 12 = 3; mean(w'/w) = 2; std([2, 4, 6]) = sqrt(8/3)
    assert xs[0] == 3.0
    assert math.isclose(err[0], 0.5 * 2 + 10.0 * math.sqrt(8.0 / 3.0), rel_tol=1e-15)
    assert not bad[0]


def test_identity_card_keeps_sigma():
    w = np.array([0.5, 1.5, 1.0, 2.0])
    xs, err, bad = xsec.xsec(w, w, sigma=5.0, dsigma=0.2, norm=1.0)
    assert xs[0] == 5.0
    assert math.isclose(err[0], 0.2 * 1.0 + 5.0 * np.std(w), rel_tol=1e-15)


def test_zero_input_weight_counts_zero():
    xs, err, bad = xsec.xsec([0.0, 2.0], [0.0, 3.0], sigma=1.0, dsigma=0.1, norm=1.0)
    # mean(w'/w) = (0 + 1.5)/2 = 0.75; std([0, 3]) = 1.5
    assert math.isclose(err[0], 0.1 * 0.75 + 1.0 * 1.5, rel_tol=1e-15)


def test_fallback_on_nan_and_nonpositive():
    xs, err, bad = xsec.xsec([1.0, 1.0], [[np.nan, 1.0], [0.0, 0.0], [2.0, 2.0]], sigma=4.0, dsigma=0.4, norm=1.0)
    assert bad[0] and np.isnan(xs[0])
    # all-zero weights: sigma' = 0, dsigma' = 0 + 0 -> fallback, max(0/4, 4/0) = inf
    assert bad[1] and err[1] == np.inf
    # a clean card: sigma' = 4, std 0, mean ratio 2 -> dsigma' = 0.8
    assert not bad[2] and math.isclose(err[2], 0.8, rel_tol=1e-15)
    # negative weights can make the error non-positive
    xs, err, bad = xsec.xsec([1.0, 1.0], [-1.0, -1.0], sigma=4.0, dsigma=0.4, norm=2.0)
    assert bad[0] and math.isclose(err[0], 0.4 * max(-4.0 / 4.0, 4.0 / -4.0), rel_tol=1e-15)
