"""Pins of the brute-force colour algebra."""
import itertools
from fractions import Fraction

import numpy as np

from oracle import colour


def test_generators():
    t = colour.T
    for a in range(8):
        np.testing.assert_allclose(t[a], t[a].conj().T, atol=1e-15)
        assert abs(np.trace(t[a])) < 1e-15
        for b in range(8):
            np.testing.assert_allclose(np.trace(t[a] @ t[b]), 0.5 * (a == b), atol=1e-15)


def test_structure_constants():
    # tabulated nonzero f^{abc} of SU(3) (1-based labels)
    table = {(1, 2, 3): 1.0, (1, 4, 7): 0.5, (1, 5, 6): -0.5, (2, 4, 6): 0.5, (2, 5, 7): 0.5,
             (3, 4, 5): 0.5, (3, 6, 7): -0.5, (4, 5, 8): np.sqrt(3) / 2, (6, 7, 8): np.sqrt(3) / 2}
    f = np.zeros((8, 8, 8))
    for (a, b, c), v in table.items():
        for (x, y, z), sgn in (((a, b, c), 1), ((b, c, a), 1), ((c, a, b), 1),
                               ((b, a, c), -1), ((a, c, b), -1), ((c, b, a), -1)):
            f[x - 1, y - 1, z - 1] = sgn * v
    t = colour.T
    for a in range(8):
        for b in range(8):
            np.testing.assert_allclose(t[a] @ t[b] - t[b] @ t[a],
                                       1j * np.einsum("c,cij->ij", f[a, b], t), atol=1e-14)


def test_one_and_two_gluon_matrices():
    np.testing.assert_allclose(colour.colour_matrix(1), [[4.0]], atol=1e-13)
    np.testing.assert_allclose(colour.colour_matrix(2), np.array([[16, -2], [-2, 16]]) / 3, atol=1e-13)


def test_four_gluon_matrix():
    c = colour.colour_matrix(4)
    assert c.shape == (24, 24)
    assert np.max(np.abs(c.imag)) < 1e-12
    c = c.real
    np.testing.assert_allclose(c, c.T, atol=1e-13)
    # diagonal: N_c C_F^4 = 3 (4/3)^4 = 256/27
    np.testing.assert_allclose(np.diag(c), 256 / 27, rtol=1e-13)
    num = 54 * c
    np.testing.assert_allclose(num, np.rint(num), atol=1e-10)
    assert set(np.rint(num).astype(int).ravel()) <= {512, 80, 71, 62, 8, -1, -10, -28, -64}
    ev = np.linalg.eigvalsh(c)
    assert ev.min() > 3.8 and ev.max() < 14.9


def test_colour_sum_against_fierz_for_two_strings():
    # sum_a (t^a t^a)_{ij} = C_F delta_ij; Tr over two-gluon strings by Fierz:
    # Tr(t^a t^b t^b t^a) = N C_F^2 = 16/3, Tr(t^a t^b t^a t^b) = -C_F/2 = -2/3
    t = colour.T
    cf = sum(t[a] @ t[a] for a in range(8))
    np.testing.assert_allclose(cf, float(Fraction(4, 3)) * np.eye(3), atol=1e-14)
    x = sum(np.trace(t[a] @ t[b] @ t[a] @ t[b]) for a, b in itertools.product(range(8), repeat=2))
    assert abs(x - (-2 / 3)) < 1e-13
