"""Colour matrices by brute force over explicit SU(3) generators, FP64.

Basis for one quark line with n gluons: the n! strings
T(pi)_{ij} = (t^{a_pi(1)} ... t^{a_pi(n)})_{ij}, i the colour of the outgoing
quark, j that of the outgoing antiquark, t^a = lambda^a / 2 (Gell-Mann).
The colour matrix is C[pi, pi'] = sum over all a's, i, j of
conj(T(pi)_{ij}) T(pi')_{ij}, summed here term by term with 3x3 matrices.

Pinned by: hermiticity, Tr(t^a t^b) = delta^{ab}/2, [t^a, t^b] = i f^{abc} t^c
with the tabulated structure constants, C for one gluon equal to C_F N_c = 4,
C for two gluons equal to [[16, -2], [-2, 16]]/3 (textbook), and the diagonal
N_c C_F^n (tests/test_oracle_colour.py).
"""
from __future__ import annotations

import itertools

import numpy as np


def gell_mann() -> np.ndarray:
    lam = np.zeros((8, 3, 3), dtype=complex)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


T = gell_mann() / 2.0


def string_tensor(perm, n):
    """T(perm) as an array [8]*n + [3, 3]; axis k is the colour of gluon k."""
    out = np.eye(3, dtype=complex).reshape((1,) * n + (3, 3))
    for slot in perm:
        shape = [1] * n + [3, 3]
        shape[slot] = 8
        out = out @ T.reshape(shape)
    return np.broadcast_to(out, (8,) * n + (3, 3))


def orderings(n):
    return list(itertools.permutations(range(n)))


def colour_matrix(n):
    """C[pi, pi'] over the n! orderings (itertools order)."""
    perms = orderings(n)
    flat = np.stack([string_tensor(p, n).reshape(-1) for p in perms])
    return np.conj(flat) @ flat.T
