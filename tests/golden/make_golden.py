"""Write tests/golden/me2_oracle.json: the oracle's |M|^2 and w' for the first
events of each seeded workload (python tests/golden/make_golden.py).

The paper prints no worked numerical example for these matrix elements, so
the stored values are the oracle's (this script calls only oracle/ and the
seeded inputs of synth/; nothing comes from the device path).  They record
the oracle's output so that a change to it shows up as a failed comparison,
and give the GPU tests a reference that needs no oracle evaluation.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth                                   # noqa: E402
from oracle import reweight                    # noqa: E402

CASES = (("ee_mumu", synth.ORIG_EW, synth.NEW_EE, 8),
         ("uu_eeg", synth.ORIG_EW, synth.NEW_UU, 8),
         ("gg_ttgg", synth.ORIG_QCD, synth.NEW_QCD, 6),
         ("gg_tttt", synth.ORIG_QCD, synth.NEW_QCD, 3))


def compute():
    out = {"note": "oracle |M|^2 (original and new card) and w' (w = 1) for the first n events of "
                   "synth.events(process, n) with the default seeds", "cases": []}
    for proc, orig, new, n in CASES:
        p = synth.events(proc, n)
        w = [1.0] * n
        wn, me0, mk = reweight.reweight(proc, p, w, orig, [new])
        me1 = mk[0]
        out["cases"].append({"process": proc, "events": n, "orig": orig.row(proc).tolist(),
                             "new": new.row(proc).tolist(), "me2_orig": [float(x) for x in me0],
                             "me2_new": [float(x) for x in me1], "w_new": [float(x) for x in wn[0]]})
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "me2_oracle.json"), "w") as f:
        json.dump(compute(), f, indent=1)
