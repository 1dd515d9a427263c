"""Symbolic SU(3) colour algebra for one quark line with gluons.

A colour factor is a dict {tuple of gluon leg ids: complex coefficient}
meaning sum_c coeff * (t^{a_c1} t^{a_c2} ...)_{ij}, with i the colour index at
the quark line's row (bar-spinor) end and j the one at its column end.

* Gluon tree attached to the quark line: f^{abe} t^e = -i [t^a, t^b] reduces
  every structure constant to commutators of generator strings.
* Colour matrix: C[s, s'] = Tr(T(s)^dagger T(s')) summed over all gluon
  indices, reduced exactly by the Fierz identity
  sum_a t^a_{ij} t^a_{kl} = 1/2 (delta_il delta_kj - 1/N delta_ij delta_kl).
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache

NC = 3


def leaf(a):
    return {(a,): 1}


def product(x, y):
    out = {}
    for kx, vx in x.items():
        for ky, vy in y.items():
            k = kx + ky
            out[k] = out.get(k, 0) + vx * vy
    return {k: v for k, v in out.items() if v != 0}


def add(x, y, sy=1):
    out = dict(x)
    for k, v in y.items():
        out[k] = out.get(k, 0) + sy * v
    return {k: v for k, v in out.items() if v != 0}


def scale(x, s):
    return {k: v * s for k, v in x.items() if v * s != 0}


def commutator(x, y):
    return add(product(x, y), product(y, x), -1)


def three_gluon(c1, c2):
    """Colour of f^{e e1 e2} with e the leg towards the quark line."""
    return scale(commutator(c1, c2), -1j)


def four_gluon(term, c1, c2, c3):
    """Colour of the three f f structures of the four-gluon vertex with legs
    (e towards the quark line, 1, 2, 3):
    0: f^{e1x} f^{23x} -> -[c1, [c2, c3]]
    1: f^{e2x} f^{13x} -> -[c2, [c1, c3]]
    2: f^{e3x} f^{12x} -> -[c3, [c1, c2]]"""
    a, b, c = [(c1, c2, c3), (c2, c1, c3), (c3, c1, c2)][term]
    return scale(commutator(a, commutator(b, c)), -1)


# ----------------------------------------------------------------- traces
def _canon(traces):
    """Relabel generator symbols in order of appearance; sort traces."""
    traces = sorted(tuple(t) for t in traces)
    mapping = {}
    out = []
    for t in traces:
        out.append(tuple(mapping.setdefault(s, len(mapping)) for s in t))
    return tuple(sorted(out))


@lru_cache(maxsize=None)
def trace_product(traces) -> Fraction:
    """Value of a product of traces of generator words in which every symbol
    appears exactly twice in total."""
    traces = [t for t in traces]
    coef = Fraction(1)
    rest = []
    for t in traces:
        if len(t) == 0:
            coef *= NC
        elif len(t) == 1:
            return Fraction(0)
        else:
            rest.append(t)
    if not rest:
        return coef
    # pick the first symbol of the first trace and find its partner
    t0 = rest[0]
    s = t0[0]
    for idx, t in enumerate(rest):
        positions = [i for i, x in enumerate(t) if x == s]
        if idx == 0 and len(positions) == 2:
            i, j = positions
            a, b = t[i + 1:j], t[j + 1:] + t[:i]
            others = rest[1:]
            # Tr(t^s A t^s B) = 1/2 Tr(A) Tr(B) - 1/(2N) Tr(A B)
            v = Fraction(1, 2) * trace_product(_canon(others + [a, b])) \
                - Fraction(1, 2 * NC) * trace_product(_canon(others + [a + b]))
            return coef * v
        if idx > 0 and positions:
            j = positions[0]
            a = t0[1:]                       # Tr(t^s A)
            b = t[j + 1:] + t[:j]            # Tr(t^s B)
            others = rest[1:idx] + rest[idx + 1:]
            # Tr(t^s A) Tr(t^s B) = 1/2 Tr(A B) - 1/(2N) Tr(A) Tr(B)
            v = Fraction(1, 2) * trace_product(_canon(others + [a + b])) \
                - Fraction(1, 2 * NC) * trace_product(_canon(others + [a, b]))
            return coef * v
    raise ValueError("unpaired generator symbol")


def colour_matrix(basis):
    """C[s, s'] = sum over indices of conj(T(s)_{ij}) T(s')_{ij} for generator
    strings s (tuples of gluon ids) = Tr(reverse(s) s')."""
    n = len(basis)
    out = [[Fraction(0)] * n for _ in range(n)]
    for i, s in enumerate(basis):
        for j, sp in enumerate(basis):
            word = tuple(reversed(s)) + tuple(sp)
            out[i][j] = trace_product(_canon([word]))
    return out
