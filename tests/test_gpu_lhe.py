"""A reweighting run on an event file (paper_2510_05100_amd.lhe.reweight_lhe):
every supported process's events reweighted on the GPU for every set of a
reweighting card, the others given weight 0, checked event by event against
the oracle (plain LHE reader + FP64 matrix elements).

Tolerances: as the full path against the oracle, 1e-12 (e+ e- -> mu+ mu-),
1e-11 (u u~ -> e+ e- g), 1e-10 (g g > t t~ g g); the weights are written with
17 significant digits, so the file adds no error.
"""
import dataclasses

import numpy as np
import pytest

import synth
from oracle import lhe as olhe
from oracle import reweight
from synth import lhe as slhe

pytestmark = pytest.mark.gpu

CARD = """launch rwgt_name=mz
set MASS 23 91.5
set DECAY 23 2.6
launch rwgt_name=as
set SMINPUTS 3 0.130
launch rwgt_name=sw
set RWGTEW 1 0.2312
"""
ORIG = synth.ORIG_EW
NEW = {"mz": dataclasses.replace(ORIG, MZ=91.5, WZ=2.6), "as": dataclasses.replace(ORIG, aS=0.130),
       "sw": dataclasses.replace(ORIG, sw2=0.2312)}
KEYS = {"e+ e- > mu+ mu-": ("ee_mumu", 1e-12), "u u~ > e+ e- g": ("uu_eeg", 1e-11),
        "g g > t t~ g g": ("gg_ttgg", 1e-10)}


@pytest.mark.parametrize("factored", [False, True])
def test_reweight_lhe_against_oracle(tmp_path, factored):
    print(f"[case] lhe run factored={factored}", flush=True)
    from gpu_util import torch_cuda
    torch_cuda()
    from paper_2510_05100_amd import lhe
    text, truth = slhe.lhe_text(n_per_process=(60, 50, 25, 15), seed=4200)
    src, dst = tmp_path / "in.lhe", tmp_path / "out.lhe"
    src.write_text(text)
    summary = lhe.reweight_lhe(src, dst, ORIG.slha(), CARD, factored=factored)
    assert summary["weights"] == ["mz", "as", "sw"]
    assert summary["processes"] == {"e+ e- > mu+ mu-": 60, "u u~ > e+ e- g": 50, "g g > t t~ g g": 25}
    out = olhe.read(dst.read_text())
    assert len(out) == len(truth)
    for proc, (key, tol) in KEYS.items():
        rows = [i for i, e in enumerate(out) if olhe.match(e, proc) is not None]
        p = np.array([olhe.momenta(out[i], proc) for i in rows])
        w = np.array([out[i]["info"][0] for i in rows])
        cards = [NEW[n] for n in ("mz", "as", "sw")]
        ref, _, _ = reweight.reweight(key, p, w, ORIG, cards)
        got = np.array([[out[i]["weights"][n] for i in rows] for n in ("mz", "as", "sw")])
        err = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)
        print(f"{key}: max rel err {err.max():.3g}", flush=True)
        assert err.max() < tol
    others = [e for e in out if all(olhe.match(e, pr) is None for pr in KEYS)]
    assert len(others) == 15 and all(e["weights"]["mz"] == 0.0 == e["weights"]["sw"] for e in others)


def test_reweight_lhe_running_alphas(tmp_path):
    """Per-event strong coupling from the file: the event's AQCDUP for the
    original card and each card's alpha_s run to the event's SCALUP."""
    print("[case] lhe run running alpha_s", flush=True)
    from gpu_util import torch_cuda
    torch_cuda()
    from oracle import running
    from paper_2510_05100_amd import lhe
    text, _ = slhe.lhe_text(n_per_process=(10, 20, 12, 3), seed=4300)
    src, dst = tmp_path / "in.lhe", tmp_path / "out.lhe"
    src.write_text(text)
    lhe.reweight_lhe(src, dst, ORIG.slha(), CARD, running_alphas=True)
    out = olhe.read(dst.read_text())
    proc = "g g > t t~ g g"
    rows = [e for e in out if olhe.match(e, proc) is not None]
    for e in rows:
        xw, scale, _, aqcd = e["info"]
        want = xw * (running.alphas(0.130, scale) / aqcd) ** 4
        assert abs(e["weights"]["as"] / want - 1) < 1e-12
        assert abs(e["weights"]["mz"] / (xw * (running.alphas(0.118, scale) / aqcd) ** 4) - 1) < 1e-12
