"""Seeded synthetic Les Houches event files (LHE v3) for the event-file tests.

A file mixes events of the three processes (and of one process the library
does not evaluate, d d~ > e+ e-) in a shuffled order.  Within each event the
incoming and the outgoing partons are written in a random order, numbers use
the usual generator formatting (explicit '+' signs, 'E' exponents, some with
Fortran 'D' exponents), and some events carry comments, an <mgrwt> block or
an existing <rwgt> block, so that a reader has to sort and match partons by
PDG code and status rather than by position.  Momenta come from
``synth.events`` (written with 17 significant digits, so they are exact).
The module holds none of the matrix-element arithmetic.
"""
from __future__ import annotations

import numpy as np

from .workloads import ORIG_EW, ORIG_QCD, events

PDG = {"ee_mumu": ([-11, 11], [-13, 13]), "uu_eeg": ([2, -2], [-11, 11, 21]),
       "gg_ttgg": ([21, 21], [6, -6, 21, 21])}
MASS = {6: 173.0, -6: 173.0}
SEED_LHE = 4000

HEADER = """<LesHouchesEvents version="3.0">
<header>
<MGVersion>
# synthetic sample for the reweighting tests
</MGVersion>
<slha>
{slha}
</slha>
{initrwgt}</header>
<init>
2212 2212 6.500000e+03 6.500000e+03 0 0 247000 247000 -4 3
+1.2500000e+01 +3.0000000e-01 +1.0000000e+00 1
+4.0000000e+00 +1.0000000e-01 +1.0000000e+00 2
+7.5000000e-01 +5.0000000e-02 +1.0000000e+00 3
<generator name='synth' version='1'>seeded</generator>
</init>
"""

PREVIOUS_RWGT = """<initrwgt>
<weightgroup name='previous' weight_name_strategy='includeIdInWeightName'>
<weight id='old_1'> set param_card mass 23 91.0 </weight>
</weightgroup>
</initrwgt>
"""


def _num(rng, v):
    """One number in a generator-like format that still reads back exactly."""
    s = f"{v:+.16e}"
    if rng.random() < 0.1:
        s = s.replace("e", "D")
    return s


def lhe_text(n_per_process=(40, 30, 20, 10), seed=SEED_LHE, previous_rwgt=True):
    """(text, truth): the file and, per event in file order, the process key
    ('ee_mumu', 'uu_eeg', 'gg_ttgg' or 'dd_ee'), its momenta in process order
    and XWGTUP."""
    rng = np.random.default_rng(seed)
    keys = ["ee_mumu", "uu_eeg", "gg_ttgg", "dd_ee"]
    moms = {k: events(k if k != "dd_ee" else "ee_mumu", n, seed=seed + 1 + i) for i, (k, n)
            in enumerate(zip(keys, n_per_process))}
    order = [(k, j) for k, n in zip(keys, n_per_process) for j in range(n)]
    rng.shuffle(order)
    slha = ORIG_EW.slha().strip() + "\n" + ORIG_QCD.slha().strip()
    out = [HEADER.format(slha=slha, initrwgt=PREVIOUS_RWGT if previous_rwgt else "")]
    truth = []
    for k, j in order:
        p = moms[k][j]
        incoming, outgoing = PDG.get(k, ([1, -1], [-11, 11]))
        codes = [(c, -1, a) for a, c in enumerate(incoming)] + [(c, 1, len(incoming) + a) for a, c in enumerate(outgoing)]
        nin = len(incoming)
        perm = list(rng.permutation(nin)) + list(nin + rng.permutation(len(outgoing)))
        xw = float(rng.uniform(0.5, 2.0))
        lines = [f" {len(codes) + 1:d} {keys.index(k) + 1:d} {_num(rng, xw)} {_num(rng, 91.188)} "
                 f"{_num(rng, 1 / 132.507)} {_num(rng, 0.118)}"]
        # an intermediate resonance line (status 2) the reader must skip
        body = []
        for slot in perm:
            c, st, a = codes[slot]
            e, px, py, pz = p[a]
            m = MASS.get(c, 0.0)
            body.append(f" {c:8d} {st:2d} {0 if st < 0 else 1:4d} {0 if st < 0 else 2:4d} {501 + slot:4d} {0:4d} "
                        f"{_num(rng, px)} {_num(rng, py)} {_num(rng, pz)} {_num(rng, e)} {_num(rng, m)} "
                        f"0.0000e+00 {_num(rng, 9.0)}")
        ptot = p[:nin].sum(axis=0)
        body.insert(nin, f" {23:8d} {2:2d} {1:4d} {2:4d} {0:4d} {0:4d} {_num(rng, ptot[1])} {_num(rng, ptot[2])} "
                         f"{_num(rng, ptot[3])} {_num(rng, ptot[0])} {_num(rng, 100.0)} 0.0000e+00 9.0000e+00")
        lines += body
        extra = rng.random()
        tail = ""
        if extra < 0.2:
            tail = "# a comment line\n<mgrwt>\n<rscale> 0 0.91188E+02</rscale>\n</mgrwt>\n"
        elif extra < 0.5:
            tail = f"<rwgt>\n<wgt id='old_1'> {_num(rng, 0.9 * xw)} </wgt>\n</rwgt>\n"
        opening = "<event>" if rng.random() < 0.8 else "<event npLO=' -1 ' npNLO=' -1 '>"
        out.append(opening + "\n" + "\n".join(lines) + "\n" + tail + "</event>\n")
        truth.append((k, p, xw))
    out.append("</LesHouchesEvents>\n")
    return "".join(out), truth
