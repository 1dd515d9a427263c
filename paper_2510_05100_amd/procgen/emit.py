"""Emit straight-line HIP device code for one process.

For each process the generated header defines, in namespace rwgt::gen_<name>:
  NPART, NCOL, NHEL, NGOOD, GOOD[] (helicities kept), AVERAGE,
  NSUM, HELW (helicities the kernels evaluate: the first NSUM of GOOD, each
  weighted by HELW),
  CNUM[NCOL][NCOL] (integer colour-matrix numerators), CDEN,
  jamps<R>(P, hel, card, jamp)  -- colour-flow amplitudes J for one helicity,
  colour_sum<R>(jamp)           -- J^dagger C J (real), with C = CNUM / CDEN.
Helicity hel is a bit pattern, bit (NPART-1-i) set meaning helicity +1 for
particle i.  Helicities that vanish identically by the chirality of a
massless fermion line (a vector coupling keeps chirality along the line) are
dropped at generation time.

Helicity parity.  With only vector couplings, real coupling constants and
real propagators (pure QCD: no photon or Z exchange, no widths), reversing
every helicity turns each external wavefunction into the complex conjugate
of the original one up to a phase, so every colour-flow amplitude becomes
the conjugate of the original times one common phase, and the colour sum
J^dagger C J (C real) is unchanged: |M_h|^2 = |M_~h|^2 for every event.  For
such processes GOOD lists one helicity of each reversed pair first (particle
0 at -1) and the kernels evaluate those NSUM = NGOOD / 2 with weight 2.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Dict, List

from . import colour as col
from .diagrams import FERMIONS, Diagrams, Leg

SPECIES = {"e": 0, "mu": 1, "u": 2, "t": 3}


def _mass(field):
    sym = FERMIONS[field][3]
    return "cd.mt" if sym else "Massless{}"


def _nsf(leg: Leg) -> int:
    """+1: u (incoming fermion) / ubar (outgoing fermion); -1: v / vbar."""
    return -1 if leg.anti else 1


def good_helicities(d: Diagrams) -> List[int]:
    legs = d.process.legs
    n = len(legs)
    lines = [d.process.line(f) for f in {l.field for l in legs if l.is_fermion} if FERMIONS[f][3] is None]
    good = []
    for hel in range(1 << n):
        h = [1 if (hel >> (n - 1 - i)) & 1 else -1 for i in range(n)]
        ok = True
        for b, f in lines:
            if FERMIONS[b.field][3] is None:          # massless line
                if (h[b.idx] * _nsf(b) > 0) != (h[f.idx] * _nsf(f) > 0):
                    ok = False
        if ok:
            good.append(hel)
    return good


def parity_symmetric(d: Diagrams) -> bool:
    """Pure QCD: no electroweak boson exchanged (chiral Z couplings and the Z
    width break the relation between reversed helicities) and no lepton."""
    return not d.pairs and all(not l.is_fermion or FERMIONS[l.field][2] for l in d.process.legs)


def summed_helicities(d: Diagrams, good: List[int]):
    """(GOOD in kernel order, NSUM, HELW): for a parity-symmetric process the
    representatives of the reversed pairs (particle 0 at helicity -1) first."""
    if not parity_symmetric(d):
        return good, len(good), 1.0
    n = len(d.process.legs)
    full = (1 << n) - 1
    kept = set(good)
    assert all((full ^ h) in kept for h in good), "kept helicities not closed under reversal"
    first = [h for h in good if not (h >> (n - 1)) & 1]
    rest = [h for h in good if (h >> (n - 1)) & 1]
    return first + rest, len(first), 2.0


class Emitter:
    def __init__(self, d: Diagrams):
        self.d = d
        self.lines: List[str] = []
        self.cache: Dict[tuple, str] = {}
        self.kcache: Dict[tuple, str] = {}
        self.count = {"ixx": 0, "oxx": 0, "vxx": 0, "ffv_in": 0, "ffv_out": 0, "ffv_vec0": 0,
                      "ffv_vecm": 0, "vvv_vec": 0, "vvvv_vec": 0, "ffv_amp": 0, "pair_w": 0}
        self.n = 0
        self.two = d.term_lines is not None
        self.fence_every = 1                     # a scheduling fence after every k-th term
        self.nterms = 0
        self.line = (d.bleg.idx, d.fleg.idx)     # main line of the amplitude being emitted

    def lkey(self, kind, seq, line):
        """Cache key of a line current; the line is part of it when the
        process has two coloured lines."""
        return (kind, seq, line) if self.two else (kind, seq)

    def new(self, prefix):
        self.n += 1
        return f"{prefix}{self.n}"

    def emit(self, s):
        self.lines.append("  " + s)

    # momenta ------------------------------------------------------------
    def kleg(self, idx):
        return f"K{idx}"

    def ksum(self, terms):
        """Name of sum_i sign_i K_legs (terms: tuple of (sign, leg)), rebuilt
        from opaque reads of the momenta at every use (see opq)."""
        key = tuple(sorted(terms))
        name = self.new("q")
        parts = []
        for mu in range(4):
            e = ""
            for s, l in key:
                sign = s * (1 if self.d.process.legs[l].incoming else -1)
                e += (" + " if sign > 0 else " - ") + f"opq(P[{l}][{mu}])"
            e = e[3:] if e.startswith(" + ") else "-" + e[3:]
            parts.append(e)
        self.emit(f"const D {name}[4] = {{{', '.join(parts)}}};")
        return name

    # external wavefunctions ---------------------------------------------
    def ext(self, leg: Leg):
        key = ("ext", leg.idx)
        if key in self.cache:
            return self.cache[key]
        name = f"w{leg.idx}"
        # momentum through opaque reads: nothing helicity-independent of the
        # external state is hoisted out of the helicity loop and kept live
        p = f"pw{leg.idx}"
        self.emit(f"const D {p}[4] = {{{', '.join(f'opq(P[{leg.idx}][{mu}])' for mu in range(4))}}};")
        if leg.kind == "V":
            self.emit(f"const Vec<R> {name} = vxx<R>({p}, h{leg.idx}, {1 if leg.incoming else -1});")
            self.count["vxx"] += 1
        elif leg.kind == "F":
            self.emit(f"const Spinor<R> {name} = ixx<R>({p}, {_mass(leg.field)}, h{leg.idx}, {_nsf(leg)});")
            self.count["ixx"] += 1
        else:
            self.emit(f"const Spinor<R> {name} = oxx<R>({p}, {_mass(leg.field)}, h{leg.idx}, {_nsf(leg)});")
            self.count["oxx"] += 1
        self.cache[key] = name
        return name

    # attachments --------------------------------------------------------
    def block_legs(self, blk):
        if blk[0] == "glu":
            from .diagrams import tree_legs
            return tree_legs(blk[1])
        sb, sf = self.d.process.line(blk[2])
        return tuple(sorted((sb.idx, sf.idx)))

    def block_k(self, blk):
        return self.ksum(tuple((1, l) for l in self.block_legs(blk)))

    def gluon(self, t):
        """Vec name of a gluon tree current (propagator included)."""
        if t[0] == "leaf":
            return self.ext(self.d.process.legs[t[1]])
        key = ("glu", t)
        if key in self.cache:
            return self.cache[key]
        if t[0] == "line":
            # the gluon a second line emits: row and column currents of that
            # line on either side of the emission vertex, joined
            line = (t[1], t[2])
            fo, fi = self.bcur(t[3], line), self.fcur(t[4], line)
            q = self.block_k(("glu", t))
            name = self.new("v")
            self.emit(f"const Vec<R> {name} = ffv_vec0_v<R>({fo}, {fi}, cd.gqq, {q});")
            self.count["ffv_vec0"] += 1
            self.cache[key] = name
            return name
        name = self.new("g")
        if t[0] == "v3":
            j1, j2 = self.gluon(t[1]), self.gluon(t[2])
            k1 = self.block_k(("glu", t[1]))
            k2 = self.block_k(("glu", t[2]))
            self.emit(f"const Vec<R> {name} = vvv_vec<R>({j1}, {k1}, {j2}, {k2}, cd.g3);")
            self.count["vvv_vec"] += 1
        else:
            term = t[1]
            j = [self.gluon(c) for c in t[2:]]
            kk = self.block_k(("glu", t))
            self.emit(f"const Vec<R> {name} = vvvv_vec<{term}, R>({j[0]}, {j[1]}, {j[2]}, {kk}, cd.g4);")
            self.count["vvvv_vec"] += 1
        self.cache[key] = name
        return name

    def pair(self, boson, field):
        key = ("pair", boson, field)
        if key in self.cache:
            return self.cache[key]
        sb, sf = self.d.process.line(field)
        fo, fi = self.ext(sb), self.ext(sf)
        q = self.ksum(((1, sb.idx), (1, sf.idx)))
        s = SPECIES[field]
        name = self.new("v")
        if boson == "a":
            self.emit(f"const Vec<R> {name} = ffv_vec0_v<R>({fo}, {fi}, cd.a[{s}], {q});")
            self.count["ffv_vec0"] += 1
        else:
            self.emit(f"const Vec<R> {name} = ffv_vecm_c<R>({fo}, {fi}, cd.zL[{s}], cd.zR[{s}], {q}, cd.mz, cd.wz);")
            self.count["ffv_vecm"] += 1
        self.cache[key] = name
        return name

    def attach(self, blk):
        """(Vec name, coupling suffix, coupling args) of an attachment on the
        main line: suffix "v" with one kappa (vector) or "c" with kappa_L,
        kappa_R (chiral)."""
        s = SPECIES[self.d.main]
        if blk[0] == "glu":
            return self.gluon(blk[1]), "v", "cd.gqq"
        boson, field = blk[1], blk[2]
        v = self.pair(boson, field)
        if boson == "a":
            return v, "v", f"cd.a[{s}]"
        return v, "c", f"cd.zL[{s}], cd.zR[{s}]"

    # main-line currents ---------------------------------------------------
    def fcur(self, seq, line=None):
        """Column spinor: Fcur(A_j..A_k) = S(q) Gamma(A_j) Fcur(A_{j+1}..A_k)."""
        line = line or self.line
        fleg = self.d.process.legs[line[1]]
        if not seq:
            return self.ext(fleg)
        key = self.lkey("F", seq, line)
        if key in self.cache:
            return self.cache[key]
        inner = self.fcur(seq[1:], line)
        v, kind, k = self.attach(seq[0])
        legs = [fleg.idx] + [l for b in seq for l in self.block_legs(b)]
        q = self.ksum(tuple((1, l) for l in legs))
        name = self.new("f")
        self.emit(f"const Spinor<R> {name} = ffv_in_{kind}<R>({inner}, {v}, {k}, {q}, {_mass(self.d.main)});")
        self.count["ffv_in"] += 1
        self.cache[key] = name
        return name

    def bcur(self, seq, line=None):
        """Row spinor: Bcur(A_1..A_j) = Bcur(A_1..A_{j-1}) Gamma(A_j) S(q)."""
        line = line or self.line
        bleg = self.d.process.legs[line[0]]
        if not seq:
            return self.ext(bleg)
        key = self.lkey("B", seq, line)
        if key in self.cache:
            return self.cache[key]
        inner = self.bcur(seq[:-1], line)
        v, kind, k = self.attach(seq[-1])
        legs = [bleg.idx] + [l for b in seq for l in self.block_legs(b)]
        q = self.ksum(tuple((-1, l) for l in legs))
        name = self.new("b")
        self.emit(f"const Spinor<R> {name} = ffv_out_{kind}<R>({inner}, {v}, {k}, {q}, {_mass(self.d.main)});")
        self.count["ffv_out"] += 1
        self.cache[key] = name
        return name

    def wpair(self, bseq, fseq):
        """W = X + Y of a (row, column) pair shared by several amplitudes."""
        key = ("W", bseq, fseq) + ((self.line,) if self.two else ())
        if key in self.cache:
            return self.cache[key]
        fo, fi = self.bcur(bseq), self.fcur(fseq)
        name = self.new("p")
        self.emit(f"const Vec<R> {name} = pair_w<R>({fo}, {fi});")
        self.count["pair_w"] += 1
        self.cache[key] = name
        return name

    def amplitude(self, seq, colour, best, shared):
        v, kind, k = self.attach(seq[best])
        if shared:
            w = self.wpair(seq[:best], seq[best + 1:])
            self.emit(f"amp = pair_amp_v<R>({w}, {v}, {k});")
        else:
            fo = self.bcur(seq[:best])
            fi = self.fcur(seq[best + 1:])
            self.emit(f"amp = ffv_amp_{kind}<R>({fo}, {fi}, {v}, {k});")
        self.count["ffv_amp"] += 1
        for key, c in colour.items():
            idx = self.d.basis.index(key)
            c = complex(c)
            assert c.real == int(c.real) and c.imag == int(c.imag)
            re, im = int(c.real), int(c.imag)
            if im == 0:
                expr = "amp" if re == 1 else ("-amp" if re == -1 else f"amp * R({re})")
            elif re == 0:
                expr = "times_i(amp)" if im == 1 else ("times_minus_i(amp)" if im == -1 else f"times_i(amp) * R({im})")
            else:
                expr = f"amp * cx<R>{{R({re}), R({im})}}"
            self.emit(f"jamp[{idx}] = jamp[{idx}] + {expr};")
        self.emit(f"note_amp(jamp, amp, {len(colour)});")
        self.nterms += 1
        if self.nterms % self.fence_every == 0:
            self.emit("term_fence();")


def colour_matrix_ints(d: Diagrams):
    if not FERMIONS[d.main][2]:
        return [[1]], 1                       # colourless main line: no colour sum
    if d.term_lines is not None:
        rows = sorted(l.idx for l in d.process.legs if l.field == d.main and l.kind == "B")
        cols = sorted(l.idx for l in d.process.legs if l.field == d.main and l.kind == "F")
        s2 = Fraction(d.colour_scale * d.colour_scale)
        cm = [[x / s2 for x in row] for row in col.colour_matrix_two_lines(d.basis, rows, cols)]
    else:
        cm = col.colour_matrix(d.basis)
    den = 1
    for row in cm:
        for x in row:
            den = den * x.denominator // math.gcd(den, x.denominator)
    num = [[int(x * den) for x in row] for row in cm]
    for i, row in enumerate(cm):
        for j, x in enumerate(row):
            assert Fraction(num[i][j], den) == x
    return num, den


def node_deps(em: "Emitter", key):
    """Direct dependencies of a plan node."""
    d = em.d
    kind = key[0]
    if kind == "ext":
        return []
    if kind == "glu":
        t = key[1]
        if t[0] == "leaf":
            return [("ext", t[1])]
        if t[0] == "line":
            line = (t[1], t[2])
            b = ("B", t[3], line) if t[3] else ("ext", line[0])
            f = ("F", t[4], line) if t[4] else ("ext", line[1])
            return [b, f]
        kids = t[1:] if t[0] == "v3" else t[2:]
        return [("ext", c[1]) if c[0] == "leaf" else ("glu", c) for c in kids]
    if kind == "pair":
        sb, sf = d.process.line(key[2])
        return [("ext", sb.idx), ("ext", sf.idx)]
    if kind == "W":
        line = key[3] if len(key) > 3 else (d.bleg.idx, d.fleg.idx)
        extra = key[3:]
        b = ("B", key[1]) + extra if key[1] else ("ext", line[0])
        f = ("F", key[2]) + extra if key[2] else ("ext", line[1])
        return [b, f]
    seq = key[1]
    line = key[2] if len(key) > 2 else (d.bleg.idx, d.fleg.idx)
    extra = key[2:]
    if kind == "F":
        inner = ("F", seq[1:]) + extra if len(seq) > 1 else ("ext", line[1])
        return [inner, attach_key(seq[0])]
    inner = ("B", seq[:-1]) + extra if len(seq) > 1 else ("ext", line[0])
    return [inner, attach_key(seq[-1])]


def attach_key(blk):
    if blk[0] == "glu":
        t = blk[1]
        return ("ext", t[1]) if t[0] == "leaf" else ("glu", t)
    return ("pair", blk[1], blk[2])


def _vector_middle(blk):
    return blk[0] == "glu" or blk[1] == "a"


def term_line(d: Diagrams, t):
    return d.term_lines[t] if d.term_lines is not None else (d.bleg.idx, d.fleg.idx)


def plan_splits(d: Diagrams):
    """Split point per amplitude term and whether its (row, column) pair is
    shared.  First, pairs (Bcur(A_1..A_{m-1}), Fcur(A_{m+1}..)) that several
    terms with a vector-coupled middle attachment can use are taken, most
    popular first: each such term then costs one four-component dot product.
    The other terms pick the split that builds the fewest new main-line
    currents, then the one nearest the middle."""
    from collections import Counter
    options = []
    counts = Counter()
    two = d.term_lines is not None
    for t, (seq, _) in enumerate(d.terms):
        opts = {}
        for m in range(len(seq)):
            if _vector_middle(seq[m]):
                opts[(seq[:m], seq[m + 1:]) + ((term_line(d, t),) if two else ())] = m
        options.append(opts)
        counts.update(opts.keys())
    splits = [None] * len(d.terms)
    shared = [False] * len(d.terms)
    for key, c in counts.most_common():
        if c < 2:
            break
        users = [t for t in range(len(d.terms)) if splits[t] is None and key in options[t]]
        if len(users) < 2:
            continue
        for t in users:
            splits[t] = options[t][key]
            shared[t] = True
    have = set()
    for t, (seq, _) in enumerate(d.terms):
        if splits[t] is None:
            continue
        m = splits[t]
        x = (term_line(d, t),) if two else ()
        have.update(("B", seq[:j]) + x for j in range(1, m + 1))
        have.update(("F", seq[j:]) + x for j in range(m + 1, len(seq)))
    for t, (seq, _) in enumerate(d.terms):
        if splits[t] is not None:
            continue
        k = len(seq)
        x = (term_line(d, t),) if two else ()

        def missing(m):
            n = sum(("B", seq[:j]) + x not in have for j in range(1, m + 1))
            return n + sum(("F", seq[j:]) + x not in have for j in range(m + 1, k))
        m = min(range(k), key=lambda m: (missing(m), abs(m - (k - 1) / 2)))
        have.update(("B", seq[:j]) + x for j in range(1, m + 1))
        have.update(("F", seq[j:]) + x for j in range(m + 1, k))
        splits[t] = m
    return splits, shared


def term_roots(d: Diagrams, seq, m, shared=False, line=None):
    line = line or (d.bleg.idx, d.fleg.idx)
    x = (line,) if d.term_lines is not None else ()
    if shared:
        return [("W", seq[:m], seq[m + 1:]) + x, attach_key(seq[m])]
    b = ("B", seq[:m]) + x if m > 0 else ("ext", line[0])
    f = ("F", seq[m + 1:]) + x if m + 1 < len(seq) else ("ext", line[1])
    return [b, f, attach_key(seq[m])]


def schedule(em: "Emitter", splits, shared):
    """Order amplitude terms to keep few currents live: repeatedly take the
    term that adds the least live data net of what it lets die."""
    d = em.d
    closure = {}

    def clos(key):
        if key not in closure:
            s = {key}
            for c in node_deps(em, key):
                s |= clos(c)
            closure[key] = frozenset(s)
        return closure[key]

    term_nodes = []
    for t, ((seq, _), m, sh) in enumerate(zip(d.terms, splits, shared)):
        s = set()
        for r in term_roots(d, seq, m, sh, term_line(d, t)):
            s |= clos(r)
        term_nodes.append(frozenset(s))
    uses = {}
    for s in term_nodes:
        for n in s:
            uses[n] = uses.get(n, 0) + 1
    size = lambda n: 8
    computed = set()
    remaining = set(range(len(d.terms)))
    order = []
    while remaining:
        best, best_cost = None, None
        for t in remaining:
            s = term_nodes[t]
            new = s - computed
            freed = [n for n in s if uses[n] == 1]
            cost = (sum(size(n) for n in new if uses[n] > 1) - sum(size(n) for n in freed if n in computed),
                    len(new), t)
            if best_cost is None or cost < best_cost:
                best, best_cost = t, cost
        order.append(best)
        remaining.discard(best)
        computed |= term_nodes[best]
        for n in term_nodes[best]:
            uses[n] -= 1
    return refine_order(order, term_nodes)


def _live_profile(order, tn):
    """(peak, sum) of the number of currents live after each term, a current
    being live from the first to the last term that needs it."""
    first, last = {}, {}
    for pos, t in enumerate(order):
        for n in tn[t]:
            if n not in first:
                first[n] = pos
            last[n] = pos
    delta = [0] * (len(order) + 1)
    for n, f in first.items():
        delta[f] += 1
        delta[last[n] + 1] -= 1
    cur = peak = total = 0
    for pos in range(len(order)):
        cur += delta[pos]
        peak = max(peak, cur)
        total += cur
    return peak, total


def refine_order(order, term_nodes, iters=30000, seed=20251005):
    """Seeded simulated annealing on the term order (moves: take one term out
    and insert it elsewhere), minimising the peak number of live currents and
    then their average."""
    import math
    import random
    if len(order) < 8:
        return order
    ids = {}
    tn = [[ids.setdefault(n, len(ids)) for n in s] for s in term_nodes]
    rng = random.Random(seed)

    def cost(o):
        p, s = _live_profile(o, tn)
        return p * 10000 + s / len(o)
    cur = list(order)
    c_cur = cost(cur)
    best, c_best = list(cur), c_cur
    for it in range(iters):
        temp = 2000.0 * (1.0 - it / iters) + 1e-3
        i, j = rng.randrange(len(cur)), rng.randrange(len(cur))
        if i == j:
            continue
        cand = list(cur)
        cand.insert(j, cand.pop(i))
        c = cost(cand)
        if c <= c_cur or rng.random() < math.exp((c_cur - c) / temp):
            cur, c_cur = cand, c
            if c < c_best:
                best, c_best = list(cand), c
    return best


# Groups of amplitude terms per helicity.  Between groups every current is
# forgotten and rebuilt on demand (from opaque momentum reads, so nothing is
# carried across): fewer currents live at once for some recomputation.
GROUPS = {"gg_ttgg": 3, "gg_tttt": 2}
# Terms between scheduling fences in the grouped (double-precision) body: the
# scheduler may interleave the terms of one span; a fence after every term
# and no fence at all both measured slower for g g -> t t~ g g.
FENCE_EVERY = {"gg_ttgg": 20, "gg_tttt": 4}


def emit_body(d: Diagrams, groups: int, fence_every: int = 1):
    """Statements of the amplitude code with the terms split into groups."""
    em = Emitter(d)
    em.fence_every = fence_every
    splits, shared = plan_splits(d)
    order = schedule(em, splits, shared)
    cuts = {round(g * len(order) / groups) for g in range(1, groups)}
    em.emit("{  // group 1")
    for pos, t in enumerate(order):
        if pos in cuts:
            em.cache.clear()
            em.emit("}")
            em.emit("term_fence();")
            em.emit("{  // next group: currents are rebuilt from here on")
        seq, colour = d.terms[t]
        em.line = term_line(d, t)
        em.amplitude(seq, colour, splits[t], shared[t])
    em.emit("}")
    return em


def generate(d: Diagrams, groups: int | None = None) -> str:
    name = d.process.name
    legs = d.process.legs
    n = len(legs)
    em = emit_body(d, 1)
    body = em.lines
    groups = groups or GROUPS.get(d.process.name, 1)
    em_g = emit_body(d, groups, FENCE_EVERY.get(d.process.name, 1)) if groups > 1 else em
    num, den = colour_matrix_ints(d)
    good, nsum, helw = summed_helicities(d, good_helicities(d))
    ncol = len(d.basis)

    out = []
    out.append(f"// Generated by paper_2510_05100_amd.procgen for '{name}'. Do not edit.")
    out.append(f"// {d.n_diagrams} Feynman diagrams, {len(d.terms)} amplitude terms, {ncol} colour flows.")
    if d.term_lines is not None:
        out.append("// Colour basis (column leg joined to the first quark; gluon leg ids on the first and the"
                   " second quark's string, row end first): "
                   + " ".join(f"[{b[0]}; ({','.join(map(str, b[1]))}) ({','.join(map(str, b[2]))})]" for b in d.basis))
        out.append(f"// Colour coefficients times {d.colour_scale}; the colour matrix is divided accordingly.")
    else:
        out.append("// Colour basis (gluon leg ids on the main line, row end first): "
                   + " ".join("(" + ",".join(map(str, b)) + ")" for b in d.basis))
    out.append("#pragma once")
    out.append('#include "helas.h"')
    out.append('#include "card.h"')
    out.append("namespace rwgt {")
    out.append(f"namespace gen_{name} {{")
    out.append(f"constexpr int NPART = {n};")
    out.append(f"constexpr int NCOL = {ncol};")
    out.append(f"constexpr int NHEL = {1 << n};")
    out.append(f"constexpr int NGOOD = {len(good)};")
    out.append(f"constexpr int NDIAG = {d.n_diagrams};")
    out.append(f"constexpr int NAMP = {len(d.terms)};")
    out.append(f"constexpr double AVERAGE = {d.process.average!r};")
    if helw != 1.0:
        out.append("// Pure QCD: reversing every helicity leaves |M_h|^2 unchanged; the first NSUM")
        out.append("// kept helicities are one of each reversed pair, weighted by HELW.")
    out.append(f"constexpr int NSUM = {nsum};")
    out.append(f"constexpr double HELW = {helw!r};")
    out.append(f"constexpr int CDEN = {den};")
    out.append(f"static __constant__ int GOOD[NGOOD] = {{{', '.join(map(str, good))}}};")
    out.append(f"constexpr int GOOD_HOST[NGOOD] = {{{', '.join(map(str, good))}}};")
    out.append("constexpr int CNUM[NCOL][NCOL] = {")
    for row in num:
        out.append("  {" + ", ".join(map(str, row)) + "},")
    out.append("};")
    out.append("// Routine counts per helicity: " + ", ".join(f"{k} {v}" for k, v in em.count.items()))
    for k, v in em.count.items():
        out.append(f"constexpr int N_{k.upper()} = {v};")
    out.append("")
    out.append("// D is the momentum type: double on the device; an operation-counting")
    out.append("// type when the host instantiates this to count arithmetic.")
    out.append("// J indexes like cx<R>[NCOL]: a register array, or an accessor into LDS.")
    out.append("template <class R, class D, class J>")
    out.append(f"__host__ __device__ __forceinline__ void jamps(const D (&P)[{n}][4], int hel, const Card<R, D>& cd, J& jamp) {{")
    for i in range(n):
        out.append(f"  const int h{i} = ((hel >> {n - 1 - i}) & 1) ? 1 : -1;")
    out.append("  for (int c = 0; c < NCOL; ++c) jamp[c] = cx<R>{R(0), R(0)};")
    out.append("  note_reset(jamp);")
    out.append("  cx<R> amp;")
    out.extend(body)
    out.append("}")
    out.append("")
    out.append(f"// Same amplitudes with the terms in {groups} group(s), currents rebuilt in each")
    out.append("// group: fewer live registers (used for the double-precision kernel).")
    out.append("// Routine counts per helicity: " + ", ".join(f"{k} {v}" for k, v in em_g.count.items()))
    out.append("template <class R, class D, class J>")
    out.append(f"__host__ __device__ __forceinline__ void jamps_grouped(const D (&P)[{n}][4], int hel, const Card<R, D>& cd, J& jamp) {{")
    for i in range(n):
        out.append(f"  const int h{i} = ((hel >> {n - 1 - i}) & 1) ? 1 : -1;")
    out.append("  for (int c = 0; c < NCOL; ++c) jamp[c] = cx<R>{R(0), R(0)};")
    out.append("  note_reset(jamp);")
    out.append("  cx<R> amp;")
    out.extend(em_g.lines)
    out.append("}")
    out.append("")
    # colour sum: J^dagger C J = sum_i J_i^* (C J)_i, C real symmetric
    out.append("template <class R, class J>")
    out.append("__host__ __device__ __forceinline__ R colour_sum(const J& jamp) {")
    out.append("  R me = R(0);")
    for i in range(ncol):
        tr = [f"R({num[i][i]}) * jamp[{i}].re"] + [f"R({2 * num[i][j]}) * jamp[{j}].re" for j in range(i + 1, ncol) if num[i][j]]
        ti = [f"R({num[i][i]}) * jamp[{i}].im"] + [f"R({2 * num[i][j]}) * jamp[{j}].im" for j in range(i + 1, ncol) if num[i][j]]
        out.append(f"  {{ const R zr = {' + '.join(tr)};")
        out.append(f"    const R zi = {' + '.join(ti)};")
        out.append(f"    me += jamp[{i}].re * zr + jamp[{i}].im * zi; }}")
    out.append(f"  return me * R(1.0 / {den}.0);")
    out.append("}")
    out.append(f"}}  // namespace gen_{name}")
    out.append("}  // namespace rwgt")
    return "\n".join(out) + "\n"
