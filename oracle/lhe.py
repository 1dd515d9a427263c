"""Plain reader of Les Houches event files (test infrastructure).

Follows the LHE format (Alwall et al., hep-ph/0609017, and its version 3
weight blocks) and the paper's Rex section: an event is the <event> block's
first data line (NUP IDPRUP XWGTUP SCALUP AQEDUP AQCDUP) and NUP particle lines
(IDUP ISTUP MOTHUP1 MOTHUP2 ICOLUP1 ICOLUP2 PUP1..5 VTIMUP SPINUP, PUP =
(px, py, pz, E, m)); events belong to a process when their external partons
(ISTUP -1 incoming, +1 outgoing) are the process's particles; each slot of
the process string takes the first unused parton with its status and PDG
code, in file order.  Added weights are <wgt id='...'> entries of the event's
<rwgt> block and <weight id='...'> entries of the header's <initrwgt>.
Pure Python (regular expressions and float()), no shared code with the
library.  Pinned by files written from known momenta and weights
(tests/test_lhe.py).
"""
from __future__ import annotations

import re

PDG = {"d": 1, "u": 2, "s": 3, "c": 4, "b": 5, "t": 6, "d~": -1, "u~": -2, "s~": -3, "c~": -4, "b~": -5,
       "t~": -6, "e-": 11, "e+": -11, "ve": 12, "ve~": -12, "mu-": 13, "mu+": -13, "vm": 14, "vm~": -14,
       "ta-": 15, "ta+": -15, "vt": 16, "vt~": -16, "g": 21, "a": 22, "z": 23, "w+": 24, "w-": -24, "h": 25}

EVENT = re.compile(r"<event(?:\s[^>]*)?>(.*?)</event>", re.S)
WGT = re.compile(r"<wgt\s+id=['\"]([^'\"]+)['\"]\s*>\s*([^<\s]+)\s*</wgt>")
WEIGHT = re.compile(r"<weight\s+id=['\"]([^'\"]+)['\"][^>]*>(.*?)</weight>", re.S)


def _f(tok):
    return float(tok.replace("D", "e").replace("d", "e"))


def read(text):
    """List of events: dict(nup, idprup, info=(xwgt, scale, aqed, aqcd),
    particles=[(id, status, E, px, py, pz)], weights={id: value})."""
    out = []
    for m in EVENT.finditer(text[text.index("</init>"):]):
        body = m.group(1)
        lines = [ln for ln in body.split("\n") if ln.strip() and not ln.strip().startswith("#")]
        head = lines[0].split()
        nup = int(head[0])
        parts = []
        for ln in lines[1:1 + nup]:
            t = ln.split()
            px, py, pz, e = (_f(x) for x in t[6:10])
            parts.append((int(t[0]), int(t[1]), e, px, py, pz))
        weights = {k: _f(v) for k, v in WGT.findall(body)}
        out.append({"nup": nup, "idprup": int(head[1]), "info": tuple(_f(x) for x in head[2:6]),
                    "particles": parts, "weights": weights})
    return out


INIT = re.compile(r"<init[\s>]")


def header_weights(text):
    """{id: description} of the header's <weight> entries."""
    head = text[:INIT.search(text).start()]
    return {k: v.strip() for k, v in WEIGHT.findall(head)}


def slots(process):
    incoming, outgoing = process.split(">")
    return [(-1, PDG[t]) for t in incoming.split()] + [(1, PDG[t]) for t in outgoing.split()]


def match(event, process):
    """Particle indices of the event in process order, or None."""
    want = slots(process)
    ext = [i for i, q in enumerate(event["particles"]) if q[1] in (-1, 1)]
    if len(ext) != len(want):
        return None
    used = set()
    idx = []
    for st, code in want:
        hit = next((i for i in ext if i not in used and event["particles"][i][1] == st
                    and event["particles"][i][0] == code), None)
        if hit is None:
            return None
        used.add(hit)
        idx.append(hit)
    return idx


def momenta(event, process):
    """[(E, px, py, pz)] in process order."""
    return [event["particles"][i][2:] for i in match(event, process)]
