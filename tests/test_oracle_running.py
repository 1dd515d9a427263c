"""Pins of the one-loop running coupling (oracle/running.py)."""
import numpy as np

from oracle import running


def test_reference_value_and_rge():
    assert running.alphas(0.118, running.MZ_REF) == 0.118
    mu = np.geomspace(5.0, 5000.0, 23)
    h = 1e-5
    a = running.alphas(0.118, mu)
    # d alpha / d ln mu^2 by central differences in t = ln mu^2 (t +- h)
    up = running.alphas(0.118, mu * np.exp(h / 2))
    dn = running.alphas(0.118, mu * np.exp(-h / 2))
    np.testing.assert_allclose((up - dn) / (2 * h), -running.b0() * a * a, rtol=1e-7)
    np.testing.assert_allclose(running.b0(), 23.0 / (12.0 * np.pi), rtol=1e-15)


def test_composition_and_asymptotic_freedom():
    a1 = running.alphas(0.130, 350.0)
    np.testing.assert_allclose(running.alphas(a1, 1200.0, mu_ref=350.0), running.alphas(0.130, 1200.0), rtol=1e-14)
    a = running.alphas(0.118, np.array([10.0, 91.1876, 1000.0]))
    assert a[0] > a[1] > a[2]
