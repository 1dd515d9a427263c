"""Tree-level QCD amplitudes with explicit colour: the colour-dressed
Berends-Giele recursion, FP64.  Test infrastructure only.

Every external colour index stays an open tensor index: off-shell currents
are built for every subset of the external legs from the textbook Feynman
rules (Peskin & Schroeder fig. 16.7, Feynman gauge):

  quark-gluon vertex      i g gamma^mu (t^a)_{ij}
  three-gluon vertex      g f^{abc} [g^{mu nu}(k1 - k2)^rho + g^{nu rho}(k2 - k3)^mu + g^{rho mu}(k3 - k1)^nu]
  four-gluon vertex       -i g^2 [f^{abe} f^{cde} (g^{mu rho} g^{nu sigma} - g^{mu sigma} g^{nu rho})
                                  + f^{ace} f^{bde} (g^{mu nu} g^{rho sigma} - g^{mu sigma} g^{nu rho})
                                  + f^{ade} f^{bce} (g^{mu nu} g^{rho sigma} - g^{mu rho} g^{nu sigma})]
  gluon propagator        -i g_{mu nu} / k^2
  quark propagator        i (q-slash + m) / (q^2 - m^2), q along the fermion arrow

(all vertex momenta incoming), with t^a = lambda^a / 2 and f^{abc} = -2 i
Tr([t^a, t^b] t^c).  Momenta k flow into the diagram from each leg: an
incoming particle brings +p, an outgoing one -p.  Fermion lines run from a
column end (u of an incoming quark or v of an outgoing antiquark) to a row
end (ubar of an outgoing quark or vbar of an incoming antiquark).  A current
over a subset S of legs is one of: a gluon current (no open fermion end), the
column current of a line (its column end in S, its row end not) or the row
current of a line (the reverse).  Currents are built from every way of
splitting S into two (three for the four-gluon vertex) smaller currents that
a vertex joins; the amplitude closes the first line's column current over
all other legs (without its propagator) on that line's row spinor.  This
sums every tree diagram once, without listing diagrams.

Identical quarks: the amplitude of each assignment of quark ends to lines
(a "pairing") is computed as for distinct flavours, and the pairings are
added with the signs of the permutations of the fermion fields (Fermi
statistics): for two lines, A = A(first pairing) - A(second pairing).

Pinned by (tests/test_oracle_dressed.py): the closed forms of u u~ -> u u~
and u u -> u u (massless, identical quarks: the exchange interference and
its sign), u u~ -> t t~ and g g -> t t~; g g -> t t~ g g against the
colour-ordered recursion of ``qcd_bg`` (a different algorithm); gauge
invariance of g g -> t t~ t t~ (a gluon's polarisation replaced by its
momentum gives zero for every colour and helicity); Lorentz invariance; Bose
symmetry of the two gluons; the exact alpha_s^4 scaling.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

from .colour import T
from .lorentz import GAMMA as _GAMMA_UP       # gamma^mu, upper index
from .lorentz import METRIC, bar, helicity_combinations, mdot, polarisation, slash, u_spinor, v_spinor

# f^{abc} = -2 i Tr([t^a, t^b] t^c)
_COMM = np.einsum("aij,bjk->abik", T, T) - np.einsum("bij,ajk->abik", T, T)
F = np.real(-2j * np.einsum("abij,cji->abc", _COMM, T))
ID4 = np.eye(4, dtype=complex)


def _es(spec, *ops):
    """einsum with contraction-order optimisation (constant colour / Dirac tensors)."""
    return np.einsum(spec, *ops, optimize=True)


def _bein(spec, x, y):
    """Two-operand einsum whose first index n (events) is shared by both
    operands and the output, as a batched matrix product over n: indices of
    both inputs missing from the output are contracted, the others are free."""
    ins, out = spec.split("->")
    sx, sy = ins.split(",")
    assert sx[0] == sy[0] == out[0] == "n"
    con = [c for c in sx[1:] if c in sy and c not in out]
    fx = [c for c in sx[1:] if c not in con]
    fy = [c for c in sy[1:] if c not in con]
    assert not set(fx) & set(fy) and sorted(fx + fy) == sorted(out[1:])
    dx = {c: x.shape[sx.index(c)] for c in sx}
    dy = {c: y.shape[sy.index(c)] for c in sy}
    xt = np.transpose(x, [0] + [sx.index(c) for c in fx] + [sx.index(c) for c in con])
    yt = np.transpose(y, [0] + [sy.index(c) for c in con] + [sy.index(c) for c in fy])
    nx, ny, nc = (int(np.prod([dx[c] for c in fx])), int(np.prod([dy[c] for c in fy])),
                  int(np.prod([dx[c] for c in con])))
    r = np.matmul(xt.reshape(x.shape[0], nx, nc), yt.reshape(y.shape[0], nc, ny))
    r = r.reshape([x.shape[0]] + [dx[c] for c in fx] + [dy[c] for c in fy])
    have = ["n"] + fx + fy
    return np.transpose(r, [have.index(c) for c in out])


@dataclasses.dataclass(frozen=True)
class Leg:
    kind: str        # "g", "q" (quark) or "qb" (antiquark)
    incoming: bool
    mass: float = 0.0

    @property
    def end(self):
        """'V' gluon, 'row' (ubar / vbar) or 'col' (u / v)."""
        if self.kind == "g":
            return "V"
        quark_like = (self.kind == "q") == (not self.incoming)    # outgoing quark or incoming antiquark
        return "row" if quark_like else "col"


@dataclasses.dataclass
class Current:
    kind: str                 # "g", or ("col", line) / ("row", line)
    legs: Tuple[int, ...]     # sorted leg indices; one colour axis each, in this order
    arr: np.ndarray           # [N, *colour(legs), own colour, 4]
    k: np.ndarray             # [N, 4] momentum flowing in from the legs


_LETTERS = "ABCDEFGHIJKLM"


def _axes(legs):
    return "".join(_LETTERS[l] for l in legs)


def _merge(*legsets):
    out = tuple(sorted(itertools.chain(*legsets)))
    assert len(set(out)) == len(out)
    return out


def _gluon_prop(k, arr):
    return (-1j / mdot(k, k))[(slice(None),) + (None,) * (arr.ndim - 1)] * arr


def _quark_prop(q, m):
    """i (q-slash + m) / (q^2 - m^2), [N, 4, 4]."""
    return 1j * (slash(q) + m * ID4) / (mdot(q, q) - m * m)[:, None, None]


def _lower(j):
    """J_mu from J^mu (last axis)."""
    return j * np.diag(METRIC)


def v3_current(a: Current, b: Current, gs):
    """Gluon current from two gluon currents (three-gluon vertex, before the propagator)."""
    ka, kb = a.k, b.k
    la, lb = _axes(a.legs), _axes(b.legs)
    legs = _merge(a.legs, b.legs)
    lo = _axes(legs)
    # bilinear pieces, colour axes x (a) and y (b) still open
    dot_ab = _bein(f"n{la}xm,n{lb}ym->n{la}{lb}xy", a.arr, _lower(b.arr))
    t1 = dot_ab[..., None] * (ka - kb)[(slice(None),) + (None,) * (dot_ab.ndim - 1)]
    ca = _bein(f"n{la}xm,nm->n{la}x", _lower(a.arr), ka + 2.0 * kb)
    cb = _bein(f"n{lb}ym,nm->n{lb}y", _lower(b.arr), 2.0 * ka + kb)
    t2 = _bein(f"n{la}x,n{lb}ym->n{la}{lb}xym", ca, b.arr)
    t3 = _bein(f"n{la}xm,n{lb}y->n{la}{lb}xym", a.arr, cb)
    v = t1 + t2 - t3
    out = gs * _es(f"n{la}{lb}xym,xyz->n{lo}zm", v, F)
    return Current("g", legs, out, ka + kb)


def v4_current(a: Current, b: Current, c: Current, gs):
    """Gluon current from three gluon currents (four-gluon vertex, before the propagator)."""
    la, lb, lc = _axes(a.legs), _axes(b.legs), _axes(c.legs)
    legs = _merge(a.legs, b.legs, c.legs)
    lo = _axes(legs)
    d_ab = _bein(f"n{la}xm,n{lb}ym->n{la}{lb}xy", a.arr, _lower(b.arr))
    d_ac = _bein(f"n{la}xm,n{lc}wm->n{la}{lc}xw", a.arr, _lower(c.arr))
    d_bc = _bein(f"n{lb}ym,n{lc}wm->n{lb}{lc}yw", b.arr, _lower(c.arr))
    ff1 = _es("xye,wze->xywz", F, F)      # f^{abe} f^{cde}, d = z the off-shell leg
    ff2 = _es("xwe,yze->xywz", F, F)      # f^{ace} f^{bde}
    ff3 = _es("xze,ywe->xywz", F, F)      # f^{ade} f^{bce}
    # term 1: (J1.J3) J2 - (J2.J3) J1
    s = _bein(f"n{la}{lc}yz,n{lb}ym->n{lo}zm", _es(f"n{la}{lc}xw,xywz->n{la}{lc}yz", d_ac, ff1), b.arr)
    s = s - _bein(f"n{lb}{lc}xz,n{la}xm->n{lo}zm", _es(f"n{lb}{lc}yw,xywz->n{lb}{lc}xz", d_bc, ff1), a.arr)
    # term 2: (J1.J2) J3 - (J2.J3) J1
    s = s + _bein(f"n{la}{lb}wz,n{lc}wm->n{lo}zm", _es(f"n{la}{lb}xy,xywz->n{la}{lb}wz", d_ab, ff2), c.arr)
    s = s - _bein(f"n{lb}{lc}xz,n{la}xm->n{lo}zm", _es(f"n{lb}{lc}yw,xywz->n{lb}{lc}xz", d_bc, ff2), a.arr)
    # term 3: (J1.J2) J3 - (J1.J3) J2
    s = s + _bein(f"n{la}{lb}wz,n{lc}wm->n{lo}zm", _es(f"n{la}{lb}xy,xywz->n{la}{lb}wz", d_ab, ff3), c.arr)
    s = s - _bein(f"n{la}{lc}yz,n{lb}ym->n{lo}zm", _es(f"n{la}{lc}xw,xywz->n{la}{lc}yz", d_ac, ff3), b.arr)
    return Current("g", legs, (-1j * gs * gs) * s, a.k + b.k + c.k)


def pair_current(r: Current, c: Current, gs):
    """Gluon current from a line's row and column currents: rbar (i g gamma^mu t^a) c."""
    lr, lc = _axes(r.legs), _axes(c.legs)
    legs = _merge(r.legs, c.legs)
    lo = _axes(legs)
    gc = _es(f"mst,n{lc}jt->n{lc}jms", _GAMMA_UP, c.arr)
    v = _bein(f"n{lr}is,n{lc}jms->n{lr}{lc}ijm", r.arr, gc)
    out = (1j * gs) * _es(f"n{lr}{lc}ijm,aij->n{lo}am", v, T)
    return Current("g", legs, out, r.k + c.k)


def col_current(g: Current, c: Current, gs):
    """Column current: (i g G-slash t^a) c, before the propagator."""
    lg, lc = _axes(g.legs), _axes(c.legs)
    legs = _merge(g.legs, c.legs)
    lo = _axes(legs)
    gsl = _es(f"n{lg}am,mst->n{lg}ast", _lower(g.arr), _GAMMA_UP)
    tc = _es(f"aij,n{lc}jt->n{lc}ait", T, c.arr)
    out = (1j * gs) * _bein(f"n{lg}ast,n{lc}ait->n{lo}is", gsl, tc)
    return Current(c.kind, legs, out, g.k + c.k)


def row_current(r: Current, g: Current, gs):
    """Row current: r (i g G-slash t^a), before the propagator."""
    lr, lg = _axes(r.legs), _axes(g.legs)
    legs = _merge(r.legs, g.legs)
    lo = _axes(legs)
    gsl = _es(f"n{lg}am,mst->n{lg}ast", _lower(g.arr), _GAMMA_UP)
    rt = _es(f"n{lr}is,aij->n{lr}ajs", r.arr, T)
    out = (1j * gs) * _bein(f"n{lr}ajs,n{lg}ast->n{lo}jt", rt, gsl)
    return Current(r.kind, legs, out, r.k + g.k)


def _propagate(cur: Current, masses):
    """Apply the propagator of the off-shell line of ``cur``."""
    if cur.kind == "g":
        return Current("g", cur.legs, _gluon_prop(cur.k, cur.arr), cur.k)
    side, line = cur.kind
    m = masses[line]
    lo = _axes(cur.legs)
    if side == "col":                                   # momentum along the arrow: k
        prop = _quark_prop(cur.k, m)
        arr = _bein(f"nst,n{lo}it->n{lo}is", prop, cur.arr)
    else:                                               # row: along the arrow -k
        prop = _quark_prop(-cur.k, m)
        arr = _bein(f"n{lo}is,nst->n{lo}it", cur.arr, prop)
    return Current(cur.kind, cur.legs, arr, cur.k)


def _kind_of(subset, ends):
    """Current type of a subset: "g", ("col", line), ("row", line), or None
    (no tree current: more than one open fermion end)."""
    open_ends = []
    for line, (r, c) in enumerate(ends):
        has_r, has_c = r in subset, c in subset
        if has_r != has_c:
            open_ends.append(("row", line) if has_r else ("col", line))
    if not open_ends:
        return "g"
    return open_ends[0] if len(open_ends) == 1 else None


def _splits(subset):
    """Unordered splits of a tuple into two non-empty parts (first part holds subset[0])."""
    first, rest = subset[0], subset[1:]
    for r in range(0, len(rest)):
        for extra in itertools.combinations(rest, r):
            a = (first,) + extra
            b = tuple(x for x in rest if x not in extra)
            yield a, b


def _triples(subset):
    """Unordered partitions of a tuple into three non-empty parts."""
    for a, bc in _splits(subset):
        if len(bc) < 2:
            continue
        for b, c in _splits(bc):
            yield a, b, c


def amplitude(ext: Dict[int, Current], ends: Sequence[Tuple[int, int]], masses, gs, nlegs):
    """Colour-tensor amplitude [N, colour of leg 0, ..., leg nlegs-1] for one
    helicity assignment.  ext: external currents per leg (before any
    vertex); ends: (row leg, column leg) per fermion line; the amplitude
    closes line 0's column current on its row spinor."""
    root = ends[0][0]
    others = tuple(l for l in range(nlegs) if l != root)
    memo: Dict[Tuple[int, ...], Current] = {}

    def current(subset, amputate=False):
        if not amputate and subset in memo:
            return memo[subset]
        if len(subset) == 1:
            cur = ext[subset[0]]
            memo[subset] = cur
            return cur
        kind = _kind_of(subset, ends)
        acc = None

        def add(c):
            nonlocal acc
            acc = c if acc is None else Current(c.kind, c.legs, acc.arr + c.arr, c.k)

        for a, b in _splits(subset):
            ka, kb = _kind_of(a, ends), _kind_of(b, ends)
            if ka is None or kb is None:
                continue
            if kind == "g":
                if ka == "g" and kb == "g":
                    add(v3_current(current(a), current(b), gs))
                elif ka != "g" and kb != "g" and ka[1] == kb[1]:      # a line's two halves
                    r, c = (a, b) if ka[0] == "row" else (b, a)
                    add(pair_current(current(r), current(c), gs))
            elif kind[0] == "col":
                if ka == "g" and kb == kind:
                    add(col_current(current(a), current(b), gs))
                elif kb == "g" and ka == kind:
                    add(col_current(current(b), current(a), gs))
            else:
                if ka == "g" and kb == kind:
                    add(row_current(current(b), current(a), gs))
                elif kb == "g" and ka == kind:
                    add(row_current(current(a), current(b), gs))
        if kind == "g":
            for a, b, c in _triples(subset):
                if all(_kind_of(x, ends) == "g" for x in (a, b, c)):
                    add(v4_current(current(a), current(b), current(c), gs))
        if acc is None:
            acc = Current(kind, subset, None, None)
        if amputate:
            return acc
        cur = _propagate(acc, masses) if acc.arr is not None else acc
        memo[subset] = cur
        return cur

    x = current(others, amputate=True)                     # line 0's column current, amputated
    r = ext[root]
    lr, lx = _axes(r.legs), _axes(x.legs)
    lo = _axes(_merge(r.legs, x.legs))
    return _bein(f"n{lr}is,n{lx}is->n{lo}", r.arr, x.arr)


def external(p, legs: Sequence[Leg], hel, line_of):
    """External currents per leg for one helicity assignment: gluons as
    eps (incoming) or eps* (outgoing) with k = +-p; quark ends as spinors
    with an identity colour tensor between the leg's index and the current's
    own index."""
    n = p.shape[0]
    out = {}
    for i, leg in enumerate(legs):
        sign = 1.0 if leg.incoming else -1.0
        k = sign * p[:, i]
        if leg.end == "V":
            e = polarisation(p[:, i], hel[i])
            if not leg.incoming:
                e = np.conj(e)
            arr = _es("ab,nm->nabm", np.eye(8), e)
            out[i] = Current("g", (i,), arr, k)
        else:
            if leg.end == "col":
                s = u_spinor(p[:, i], leg.mass, hel[i]) if leg.incoming else v_spinor(p[:, i], leg.mass, hel[i])
            else:
                s = bar(v_spinor(p[:, i], leg.mass, hel[i])) if leg.incoming else bar(u_spinor(p[:, i], leg.mass, hel[i]))
            arr = _es("ij,ns->nijs", np.eye(3), s)
            out[i] = Current((leg.end, line_of[i]), (i,), arr, k)
    assert all(v.arr.shape[0] == n for v in out.values())
    return out


def me2(p, legs: Sequence[Leg], pairings, gs, average):
    """Colour- and helicity-summed |M|^2 times ``average`` per event.

    pairings: list of (sign, [(row leg, column leg) per line]) whose
    amplitudes are added with their signs (one entry for distinct flavours).
    Every helicity assignment runs in one pass: the assignments are stacked
    on the event axis (assignment-major), which the recursion treats like
    more events.
    """
    n = len(legs)
    nev = p.shape[0]
    hels = helicity_combinations(n)
    pp = np.tile(p, (len(hels), 1, 1))
    amp = None
    for sign, ends in pairings:
        line_of = {}
        for line, (r, c) in enumerate(ends):
            line_of[r] = line_of[c] = line
        masses = [legs[r].mass for r, _ in ends]
        per_hel = {}
        for lam in (-1, 1):
            per_hel[lam] = external(p, legs, [lam] * n, line_of)
        ext = {}
        for i in range(n):
            arr = np.concatenate([per_hel[h[i]][i].arr for h in hels], axis=0)
            cur = per_hel[1][i]
            ext[i] = Current(cur.kind, cur.legs, arr, np.tile(cur.k, (len(hels), 1)))
        a = sign * amplitude(ext, ends, masses, gs, n)
        amp = a if amp is None else amp + a
    sq = np.sum(np.abs(amp.reshape(amp.shape[0], -1)) ** 2, axis=1)
    del pp
    return average * sq.reshape(len(hels), nev).sum(axis=0)


def amplitude_for(p, legs: Sequence[Leg], pairings, gs, hel, gauge=None):
    """Colour-tensor amplitude for one helicity assignment (pairings added
    with their signs); gauge: a gluon leg whose polarisation is replaced by
    its momentum (scaled by 1/E), which gives zero in a gauge-invariant sum."""
    n = len(legs)
    amp = None
    for sign, ends in pairings:
        line_of = {}
        for line, (r, c) in enumerate(ends):
            line_of[r] = line_of[c] = line
        masses = [legs[r].mass for r, _ in ends]
        ext = external(p, legs, hel, line_of)
        if gauge is not None:
            k = p[:, gauge] / p[:, gauge, :1]
            ext[gauge] = Current("g", (gauge,), np.einsum("ab,nm->nabm", np.eye(8), k.astype(complex)), ext[gauge].k)
        a = sign * amplitude(ext, ends, masses, gs, n)
        amp = a if amp is None else amp + a
    return amp


# ----------------------------------------------------------- processes
def gg_tttt_legs(mt):
    return [Leg("g", True), Leg("g", True), Leg("q", False, mt), Leg("qb", False, mt),
            Leg("q", False, mt), Leg("qb", False, mt)]


# the two assignments of antitops to tops, with the sign of the exchange
GG_TTTT_PAIRINGS = [(1.0, [(2, 3), (4, 5)]), (-1.0, [(2, 5), (4, 3)])]


def me2_gg_tttt(p: np.ndarray, card) -> np.ndarray:
    """g(p0) g(p1) -> t(p2) t~(p3) t(p4) t~(p5), pure QCD at order g_s^4 in
    the amplitude: |M|^2 averaged over the incoming spins (1/4) and colours
    (1/64), times 1/(2! 2!) for the identical tops and antitops."""
    gs = math.sqrt(4.0 * math.pi * card.aS)
    average = 0.25 / 64.0 / 4.0
    return me2(p, gg_tttt_legs(card.MT), GG_TTTT_PAIRINGS, gs, average)
