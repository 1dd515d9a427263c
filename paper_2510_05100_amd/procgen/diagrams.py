"""Tree-level Feynman diagrams along one fermion line, with current reuse.

Supported class of processes: one main fermion line (row end B, column end
F) carrying an ordered sequence of attachments; an attachment is either a
gluon tree over a subset of the external gluons (main line coloured) built
from three- and four-gluon vertices, or the photon/Z current of a second,
colourless fermion pair.  This covers e+e- -> mu+mu- (2 diagrams),
u u~ -> e+e- g (4) and g g -> t t~ g g (123).

Two coloured lines of one flavour (g g -> t t~ t t~): for each assignment of
the antiquarks to the quarks (a pairing; the second enters with a minus sign,
Fermi statistics) the first quark's line is the main line, and the second
line is a leaf of one of its gluon trees: the gluon current that line emits,
with its own ordered gluon-tree attachments on either side of the emission
vertex.  Colour: the emitted gluon's generators on the two lines are joined
by the Fierz identity into the basis of products of two generator strings,
one per quark.

Each diagram is evaluated at one vertex of the main line,
amp = Bcur(A_1..A_{m-1}) Gamma(A_m) Fcur(A_{m+1}..A_k), where Bcur and Fcur
are off-shell spinors grown from the two ends; the split m is chosen greedily
to reuse currents already built.  Four-gluon vertices contribute three
amplitude terms (one per colour structure) to a single diagram.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import Dict, List, Optional, Tuple

from . import colour as col

# fermion fields: (charge, T3, coloured, mass symbol)
FERMIONS = {
    "e": (-1.0, -0.5, False, None),
    "mu": (-1.0, -0.5, False, None),
    "u": (2.0 / 3.0, 0.5, True, None),
    "t": (2.0 / 3.0, 0.5, True, "mt"),
}


@dataclasses.dataclass(frozen=True)
class Leg:
    idx: int
    field: str            # e, mu, u, t, g
    anti: bool
    incoming: bool

    @property
    def is_fermion(self):
        return self.field in FERMIONS

    @property
    def kind(self):
        """'B' row spinor, 'F' column spinor, 'V' vector."""
        if not self.is_fermion:
            return "V"
        # row end: outgoing fermion (ubar) or incoming antifermion (vbar)
        return "B" if (self.incoming == self.anti) else "F"


@dataclasses.dataclass
class Process:
    name: str
    legs: List[Leg]
    average: float        # spin/colour average times identical-particle factor

    def line(self, field):
        b = [l for l in self.legs if l.field == field and l.kind == "B"]
        f = [l for l in self.legs if l.field == field and l.kind == "F"]
        assert len(b) == 1 and len(f) == 1
        return b[0], f[0]


def parse(name: str, text: str) -> Process:
    """Build a Process from a string such as "g g > t t~ g g"."""
    lhs, rhs = [s.split() for s in text.split(">")]
    legs = []
    for inc, toks in ((True, lhs), (False, rhs)):
        for t in toks:
            anti = t.endswith("~") or t.endswith("+")
            base = t.rstrip("~+-")
            if base == "e" and t == "e-":
                anti = False
            if base == "mu" and t == "mu-":
                anti = False
            legs.append(Leg(len(legs), base, anti, inc))
    # averages: spins of the 2 incoming particles, colours, identical finals
    avg = 1.0
    for l in legs[:2]:
        avg /= 2.0
        if l.field == "g":
            avg /= 8.0
        elif l.is_fermion and FERMIONS[l.field][2]:
            avg /= 3.0
    finals = [l.field + ("~" if l.anti else "") for l in legs[2:]]
    for f in set(finals):
        n = finals.count(f)
        for k in range(2, n + 1):
            avg /= k
    return Process(name, legs, avg)


# ----------------------------------------------------------- gluon trees
def gluon_trees(subset: Tuple[int, ...]):
    """All gluon trees over a sorted tuple of gluon leg ids; each tree is
    ('leaf', a) | ('v3', t1, t2) | ('v4', term, t1, t2, t3)."""
    subset = tuple(sorted(subset))
    if len(subset) == 1:
        return [("leaf", subset[0])]
    out = []
    first, rest = subset[0], subset[1:]
    # unordered split into two: S1 contains the smallest leg
    for r in range(0, len(rest)):
        for extra in itertools.combinations(rest, r):
            s1 = (first,) + extra
            s2 = tuple(x for x in rest if x not in extra)
            for t1 in gluon_trees(s1):
                for t2 in gluon_trees(s2):
                    out.append(("v3", t1, t2))
    # unordered partitions into three blocks
    for p in set_partitions(subset, 3):
        for t1 in gluon_trees(p[0]):
            for t2 in gluon_trees(p[1]):
                for t3 in gluon_trees(p[2]):
                    for term in range(3):
                        out.append(("v4", term, t1, t2, t3))
    return out


def set_partitions(items, k):
    """Partitions of a tuple into exactly k non-empty blocks, blocks ordered
    by their smallest element."""
    items = tuple(items)
    if k == 1:
        yield (items,)
        return
    if len(items) < k:
        return
    first, rest = items[0], items[1:]
    # first block contains `first`
    for r in range(0, len(rest) - k + 2):
        for extra in itertools.combinations(rest, r):
            block = (first,) + extra
            remaining = tuple(x for x in rest if x not in extra)
            for sub in set_partitions(remaining, k - 1):
                yield (block,) + sub


def line_leaves(line, gsub):
    """Gluon currents emitted by a second fermion line (row leg, column leg)
    with the gluons gsub attached to it directly: every ordered sequence of
    gluon-tree blocks over gsub and every position of the emission vertex in
    it, as ('line', row, col, blocks before, blocks after)."""
    gsub = tuple(sorted(gsub))
    blocks = {sub: [("glu", t) for t in gluon_trees(sub)]
              for r in range(1, len(gsub) + 1) for sub in itertools.combinations(gsub, r)}
    out = []
    for seq_legs in ordered_partitions(gsub, blocks):
        for seq in itertools.product(*[blocks[k] for k in seq_legs]):
            for pos in range(len(seq) + 1):
                out.append(("line", line[0], line[1], tuple(seq[:pos]), tuple(seq[pos:])))
    return out


def gluon_trees_line(gsub, line):
    """All gluon trees over the gluons gsub and one leaf of the second line
    (line_leaves), built from three- and four-gluon vertices; the part that
    holds the line comes first at each vertex."""
    gsub = tuple(sorted(gsub))
    out = line_leaves(line, gsub)
    for r in range(1, len(gsub) + 1):
        for pure in itertools.combinations(gsub, r):
            rest = tuple(x for x in gsub if x not in pure)
            for t1 in gluon_trees_line(rest, line):
                for t2 in gluon_trees(pure):
                    out.append(("v3", t1, t2))
    for r in range(2, len(gsub) + 1):
        for pure in itertools.combinations(gsub, r):
            rest = tuple(x for x in gsub if x not in pure)
            for p1, p2 in set_partitions(pure, 2):
                for t1 in gluon_trees_line(rest, line):
                    for t2 in gluon_trees(p1):
                        for t3 in gluon_trees(p2):
                            for term in range(3):
                                out.append(("v4", term, t1, t2, t3))
    return out


def tree_legs(t):
    if t[0] == "leaf":
        return (t[1],)
    if t[0] == "line":
        return tuple(sorted((t[1], t[2]) + sum((tree_legs(b[1]) for b in t[3] + t[4]), ())))
    kids = t[1:] if t[0] == "v3" else t[2:]
    return tuple(sorted(sum((tree_legs(c) for c in kids), ())))


def tree_colour(t):
    if t[0] == "leaf":
        return col.leaf(t[1])
    if t[0] == "line":
        return col.leaf(col.X)
    if t[0] == "v3":
        return col.three_gluon(tree_colour(t[1]), tree_colour(t[2]))
    return col.four_gluon(t[1], tree_colour(t[2]), tree_colour(t[3]), tree_colour(t[4]))


def line_colour(t):
    """Colour string of a second line's leaf: its attachments with the
    emitted gluon's generator (col.X) at the emission vertex."""
    c = {(): 1}
    for blk in t[3]:
        c = col.product(c, tree_colour(blk[1]))
    c = col.product(c, col.leaf(col.X))
    for blk in t[4]:
        c = col.product(c, tree_colour(blk[1]))
    return c


def find_line(t):
    """The second line's leaf inside a gluon tree, or None."""
    if t[0] == "line":
        return t
    if t[0] == "leaf":
        return None
    kids = t[1:] if t[0] == "v3" else t[2:]
    for k in kids:
        f = find_line(k)
        if f is not None:
            return f
    return None


def canonical_tree(t):
    """The tree with every four-gluon term index set to 0 (one diagram)."""
    if t[0] == "leaf":
        return t
    if t[0] == "line":
        return t[:3] + (tuple(("glu", canonical_tree(b[1])) for b in t[3]),
                        tuple(("glu", canonical_tree(b[1])) for b in t[4]))
    if t[0] == "v3":
        return ("v3", canonical_tree(t[1]), canonical_tree(t[2]))
    return ("v4", 0, canonical_tree(t[2]), canonical_tree(t[3]), canonical_tree(t[4]))


# ---------------------------------------------------------------- diagrams
@dataclasses.dataclass
class Diagrams:
    process: Process
    main: str                                  # main-line fermion field
    bleg: Leg
    fleg: Leg
    gluons: Tuple[int, ...]
    pairs: List[Tuple[str, str]]               # (boson, secondary field)
    terms: List[Tuple[tuple, complex, Dict]]   # (block sequence, colour dict)
    basis: List[Tuple[int, ...]]
    n_diagrams: int
    # two coloured lines: the main line (row leg, column leg) of each term
    # (None: bleg, fleg for every term), and the factor that makes every
    # colour coefficient an integer
    term_lines: Optional[List[Tuple[int, int]]] = None
    colour_scale: int = 1


def couples(boson, field):
    q, _, coloured, _ = FERMIONS[field]
    if boson == "g":
        return coloured
    if boson == "a":
        return q != 0.0
    return boson == "Z"


def build(process: Process) -> Diagrams:
    fermion_fields = []
    for l in process.legs:
        if l.is_fermion and l.field not in fermion_fields:
            fermion_fields.append(l.field)
    coloured = [f for f in fermion_fields if FERMIONS[f][2]]
    if len(coloured) == 1 and sum(1 for l in process.legs if l.field == coloured[0]) == 4:
        return build_two_lines(process, coloured[0])
    main = coloured[0] if coloured else fermion_fields[0]
    assert len(coloured) <= 1, "one coloured fermion line at most"
    bleg, fleg = process.line(main)
    gluons = tuple(l.idx for l in process.legs if l.field == "g")
    secondary = [f for f in fermion_fields if f != main]
    pairs = [(b, f) for f in secondary for b in ("a", "Z") if couples(b, f) and couples(b, main)]

    # attachment blocks keyed by the legs they cover
    blocks: Dict[Tuple[int, ...], list] = {}
    if gluons:
        assert couples("g", main)
        for r in range(1, len(gluons) + 1):
            for sub in itertools.combinations(gluons, r):
                blocks[sub] = [("glu", t) for t in gluon_trees(sub)]
    for b, f in pairs:
        sb, sf = process.line(f)
        blocks.setdefault(tuple(sorted((sb.idx, sf.idx))), []).append(("pair", b, f))

    others = tuple(sorted(l.idx for l in process.legs if l.idx not in (bleg.idx, fleg.idx)))
    basis = [tuple(p) for p in itertools.permutations(gluons)] if gluons else [()]

    terms = []
    diagram_keys = set()
    for seq_legs in ordered_partitions(others, blocks):
        for seq in itertools.product(*[blocks[s] for s in seq_legs]):
            colour = {(): 1}
            for blk in seq:
                colour = col.product(colour, tree_colour(blk[1]) if blk[0] == "glu" else {(): 1})
            terms.append((seq, colour))
            diagram_keys.add(tuple(("glu", canonical_tree(b[1])) if b[0] == "glu" else b for b in seq))
    for _, colour in terms:
        for key in colour:
            assert key in basis, key
    return Diagrams(process, main, bleg, fleg, gluons, pairs, terms, basis, len(diagram_keys))


def ordered_partitions(items, blocks):
    """Ordered sequences of keys of ``blocks`` partitioning ``items``."""
    items = tuple(sorted(items))
    if not items:
        yield ()
        return
    for key in blocks:
        if set(key) <= set(items):
            rest = tuple(x for x in items if x not in key)
            for tail in ordered_partitions(rest, blocks):
                yield (key,) + tail


# ------------------------------------------------------- two coloured lines
def build_two_lines(process: Process, field: str) -> Diagrams:
    """Two lines of one coloured flavour and external gluons (no photon/Z)."""
    rows = [l for l in process.legs if l.field == field and l.kind == "B"]
    cols = [l for l in process.legs if l.field == field and l.kind == "F"]
    assert len(rows) == 2 and len(cols) == 2 and all(l.field in (field, "g") for l in process.legs)
    gluons = tuple(l.idx for l in process.legs if l.field == "g")
    r0, r1 = rows[0].idx, rows[1].idx
    # pairings: the column partner of each row; the second swaps the columns
    pairings = [(1, (cols[0].idx, cols[1].idx)), (-1, (cols[1].idx, cols[0].idx))]
    basis = []
    for partner in (cols[0].idx, cols[1].idx):
        for k in range(len(gluons) + 1):
            for on0 in itertools.permutations(gluons, k):
                rest = [g for g in gluons if g not in on0]
                for on1 in itertools.permutations(rest):
                    basis.append((partner, tuple(on0), tuple(on1)))
    terms, lines = [], []
    diagram_keys = set()
    for sign, (c0, c1) in pairings:
        main, second = (r0, c0), (r1, c1)
        blocks: Dict[Tuple[int, ...], list] = {}
        for r in range(1, len(gluons) + 1):
            for sub in itertools.combinations(gluons, r):
                blocks[sub] = [("glu", t) for t in gluon_trees(sub)]
        for r in range(0, len(gluons) + 1):
            for sub in itertools.combinations(gluons, r):
                blocks[tuple(sorted(sub + second))] = [("glu", t) for t in gluon_trees_line(sub, second)]
        others = tuple(sorted(l.idx for l in process.legs if l.idx not in main))
        for seq_legs in ordered_partitions(others, blocks):
            if not any(second[0] in k for k in seq_legs):
                continue
            for seq in itertools.product(*[blocks[k] for k in seq_legs]):
                ca = {(): 1}
                leaf = None
                for blk in seq:
                    ca = col.product(ca, tree_colour(blk[1]))
                    leaf = leaf or find_line(blk[1])
                colour = col.fierz(ca, line_colour(leaf), main, second, sign)
                terms.append((seq, colour))
                lines.append(main)
                diagram_keys.add((main, tuple(("glu", canonical_tree(b[1])) for b in seq)))
    scale = col.FIERZ_SCALE
    for _, colour in terms:
        for key in colour:
            assert key in basis, key
    bleg = process.legs[r0]
    return Diagrams(process, field, bleg, process.legs[cols[0].idx], gluons, [], terms, basis,
                    len(diagram_keys), term_lines=lines, colour_scale=scale)
