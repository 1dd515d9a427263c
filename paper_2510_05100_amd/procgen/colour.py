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
X = "x"          # the generator of a gluon joining two quark lines (contracted by fierz)


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


# ------------------------------------------------------------ two lines
def fierz(ca, cb, main, second, sign=1):
    """Colour of a product of two lines' strings joined by one gluon: ca on
    the main line (row, column), cb on the second, each holding X once.
    sum_x (U t^x V)_{i j} (P t^x Q)_{k l}
        = 1/2 (U Q)_{i l} (P V)_{k j} - 1/(2N) (U V)_{i j} (P Q)_{k l}.
    Returned times 2N (integer coefficients, times sign), keyed by (column
    joined to the main row, string on the main row, string on the second
    row)."""
    out = {}
    for sa, va in ca.items():
        ia = sa.index(X)
        u, v = sa[:ia], sa[ia + 1:]
        for sb, vb in cb.items():
            ib = sb.index(X)
            p, q = sb[:ib], sb[ib + 1:]
            for key, c in (((second[1], u + q, p + v), NC), ((main[1], u + v, p + q), -1)):
                out[key] = out.get(key, 0) + sign * va * vb * c
    return {k: v for k, v in out.items() if v != 0}


FIERZ_SCALE = 2 * NC     # fierz returns colour factors times this


def colour_matrix_two_lines(basis, rows, cols):
    """C[b, b'] = sum over all indices of conj(B_b) B_b' for basis elements
    (column joined to rows[0], string on rows[0], string on rows[1]): the
    index loops closed by following each quark line from its row to its
    column in B_b' and back through the conjugate of B_b."""
    n = len(basis)
    out = [[Fraction(0)] * n for _ in range(n)]
    for i, (p, s0, s1) in enumerate(basis):
        col_of = {rows[0]: p, rows[1]: cols[1] if p == cols[0] else cols[0]}
        row_at = {v: k for k, v in col_of.items()}
        conj = {rows[0]: tuple(reversed(s0)), rows[1]: tuple(reversed(s1))}
        for j, (pp, t0, t1) in enumerate(basis):
            colp = {rows[0]: pp, rows[1]: cols[1] if pp == cols[0] else cols[0]}
            strp = {rows[0]: t0, rows[1]: t1}
            loops, seen = [], set()
            for start in rows:
                if start in seen:
                    continue
                word, r = (), start
                while r not in seen:
                    seen.add(r)
                    word += strp[r]
                    back = row_at[colp[r]]          # the row B_b joins to that column
                    word += conj[back]
                    r = back
                loops.append(word)
            out[i][j] = trace_product(_canon(loops))
    return out
