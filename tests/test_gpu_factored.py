"""The coupling-factored path (rwgt_eval_factored) against the full
matrix-element path and the oracle.

Tolerances: the factored path rebuilds each |M|^2 from four probe
evaluations and the closed form of the couplings and the Z propagator; it
agrees with the full path to FP64 rounding amplified by cancellations between
diagrams and between the photon and Z terms, the same amplification as the
full path shows against the oracle: 1e-12 relative on w' for
e+ e- -> mu+ mu-, 1e-11 for u u~ -> e+ e- g, 1e-12 for the alpha_s scaling of
g g -> t t~ g g.  In mixed precision the probes carry the float amplitudes'
error: 2e-5 against the full mixed path.
"""
import dataclasses

import numpy as np
import pytest

import synth
from oracle import reweight

from gpu_util import PROCESS_TEXT, dev, rel_err, torch_cuda

pytestmark = pytest.mark.gpu


def _cards_ew():
    grid = synth.batch_grid()
    extra = [dataclasses.replace(synth.ORIG_EW, aEWM1=128.0), dataclasses.replace(synth.ORIG_EW, aS=0.125),
             synth.ORIG_EW, dataclasses.replace(synth.ORIG_EW, MZ=95.0, WZ=4.0, sw2=0.25)]
    return grid + extra


def _both(process, p, w, orig, cards, precision=0):
    torch = torch_cuda()
    import paper_2510_05100_amd as rw
    rows = np.stack([c.row(process) for c in cards])
    with rw.Reweighter(PROCESS_TEXT[process], orig.slha(), precision) as r:
        pd, wd = dev(p), dev(w)
        full = torch.empty((len(cards), p.shape[0]), dtype=torch.float64, device="cuda")
        fac = torch.full((len(cards), p.shape[0]), np.nan, dtype=torch.float64, device="cuda")
        r.eval(pd, wd, rows, full)
        r.eval_factored(pd, wd, rows, fac)
        torch.cuda.synchronize()
        return full.cpu().numpy(), fac.cpu().numpy()


@pytest.mark.parametrize("process,n,tol", [("ee_mumu", 2000, 1e-12), ("uu_eeg", 3000 + 17, 1e-11)])
def test_factored_matches_full_path_fp64(process, n, tol):
    print(f"[case] factored {process} n={n}", flush=True)
    p = synth.events(process, n)
    w = np.random.default_rng(6).uniform(0.5, 2.0, n)
    cards = _cards_ew() if process == "uu_eeg" else [c for c in _cards_ew() if c.aS == synth.ORIG_EW.aS]
    full, fac = _both(process, p, w, synth.ORIG_EW, cards)
    err = rel_err(fac, full)
    print(f"max rel diff {err.max():.3g}", flush=True)
    assert err.max() < tol


def test_factored_matches_oracle():
    print("[case] factored vs oracle", flush=True)
    n = 200
    p = synth.events("uu_eeg", n)
    w = np.linspace(0.3, 3.0, n)
    cards = _cards_ew()[::7]
    _, fac = _both("uu_eeg", p, w, synth.ORIG_EW, cards)
    ref, _, _ = reweight.reweight("uu_eeg", p, w, synth.ORIG_EW, cards)
    assert rel_err(fac, ref).max() < 1e-11


def test_factored_qcd_alpha_s_scaling():
    print("[case] factored gg_ttgg", flush=True)
    n = 300
    p = synth.events("gg_ttgg", n)
    cards = [synth.NEW_QCD, dataclasses.replace(synth.ORIG_QCD, aS=0.1), synth.ORIG_QCD]
    full, fac = _both("gg_ttgg", p, np.ones(n), synth.ORIG_QCD, cards)
    assert rel_err(fac, full).max() < 1e-12
    np.testing.assert_allclose(fac[0], (0.130 / 0.118) ** 4, rtol=1e-13)


def test_factored_mixed_precision():
    print("[case] factored mixed", flush=True)
    n = 2000
    p = synth.events("uu_eeg", n)
    full, fac = _both("uu_eeg", p, np.ones(n), synth.ORIG_EW, _cards_ew(), precision=1)
    assert rel_err(fac, full).max() < 2e-5


def test_factored_edge_cases():
    print("[case] factored edges", flush=True)
    torch = torch_cuda()
    import paper_2510_05100_amd as rw
    # alpha_s = 0 in the original card: every |M|^2_orig = 0 -> w' = 0
    zero = dataclasses.replace(synth.ORIG_EW, aS=0.0)
    p = synth.events("uu_eeg", 50)
    _, fac = _both("uu_eeg", p, np.ones(50), zero, [synth.NEW_UU])
    np.testing.assert_array_equal(fac, 0.0)
    with rw.Reweighter(PROCESS_TEXT["uu_eeg"], synth.ORIG_EW.slha()) as r:
        empty = torch.empty((0, 5, 4), dtype=torch.float64, device="cuda")
        r.eval_factored(empty, torch.empty(0, dtype=torch.float64, device="cuda"), synth.NEW_UU.row("uu_eeg"),
                        torch.empty((1, 0), dtype=torch.float64, device="cuda"))
    with rw.Reweighter(PROCESS_TEXT["gg_ttgg"], synth.ORIG_QCD.slha()) as r:
        q = synth.events("gg_ttgg", 3)
        out = torch.empty((1, 3), dtype=torch.float64, device="cuda")
        with pytest.raises(rw.RwgtError, match="EPARAM"):
            r.eval_factored(dev(q), dev(np.ones(3)), [0.118, 172.5], out)
