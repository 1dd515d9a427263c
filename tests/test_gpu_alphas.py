"""Reweighting with the strong coupling per event (rwgt_eval_alphas) against
the oracle evaluated with each event's own couplings.

Tolerances: as the full path against the oracle (1e-12 e+ e- -> mu+ mu-,
1e-11 u u~ -> e+ e- g); for g g > t t~ g g the ratio has the closed form
w (a_k(mu_i) / a_0(i))^4, checked to 1e-12.
"""
import dataclasses

import numpy as np
import pytest

import synth
from oracle import reweight, running

from gpu_util import PROCESS_TEXT, dev, rel_err, torch_cuda

pytestmark = pytest.mark.gpu


def _run(process, p, w, orig, cards, alphas_orig, scales):
    torch = torch_cuda()
    import paper_2510_05100_amd as rw
    rows = np.stack([c.row(process) for c in cards])
    with rw.Reweighter(PROCESS_TEXT[process], orig.slha()) as r:
        out = torch.empty((len(cards), p.shape[0]), dtype=torch.float64, device="cuda")
        rw.rwgt_set_stream(r.ctx, None)
        rw.rwgt_eval_alphas(r.ctx, dev(p), dev(w), None if alphas_orig is None else dev(alphas_orig), dev(scales),
                            rows, out)
        torch.cuda.synchronize()
        return out.cpu().numpy()


def test_uu_eeg_per_event_alpha_s_against_oracle():
    print("[case] alphas uu_eeg", flush=True)
    n = 120
    rng = np.random.default_rng(21)
    p = synth.events("uu_eeg", n)
    w = rng.uniform(0.5, 2.0, n)
    a_orig = rng.uniform(0.10, 0.13, n)
    scales = rng.uniform(50.0, 800.0, n)
    cards = [dataclasses.replace(synth.NEW_UU, aS=0.125), dataclasses.replace(synth.ORIG_EW, aS=0.110)]
    got = _run("uu_eeg", p, w, synth.ORIG_EW, cards, a_orig, scales)
    ref = np.empty_like(got)
    for i in range(n):
        o = dataclasses.replace(synth.ORIG_EW, aS=float(a_orig[i]))
        ci = [dataclasses.replace(c, aS=float(running.alphas(c.aS, scales[i]))) for c in cards]
        r, _, _ = reweight.reweight("uu_eeg", p[i:i + 1], w[i:i + 1], o, ci)
        ref[:, i] = r[:, 0]
    assert rel_err(got, ref).max() < 1e-11


def test_gg_ttgg_closed_form_and_default_original():
    print("[case] alphas gg_ttgg", flush=True)
    n = 257
    rng = np.random.default_rng(22)
    p = synth.events("gg_ttgg", n)
    w = np.ones(n)
    scales = rng.uniform(300.0, 3000.0, n)
    a_orig = running.alphas(0.118, scales)
    cards = [synth.NEW_QCD]
    got = _run("gg_ttgg", p, w, synth.ORIG_QCD, cards, a_orig, scales)
    want = (running.alphas(0.130, scales) / a_orig) ** 4
    assert rel_err(got[0], want).max() < 1e-12
    # without the events' alpha_s the original card is run to the scales: the same result
    got2 = _run("gg_ttgg", p, w, synth.ORIG_QCD, cards, None, scales)
    assert rel_err(got2[0], want).max() < 1e-12


def test_edge_cases():
    print("[case] alphas edges", flush=True)
    n = 40
    p = synth.events("ee_mumu", n)
    w = np.linspace(1, 2, n)
    scales = np.full(n, 200.0)
    # no strong coupling in e+ e- -> mu+ mu-: identical to rwgt_eval
    got = _run("ee_mumu", p, w, synth.ORIG_EW, [synth.NEW_EE], np.full(n, 0.1), scales)
    ref, _, _ = reweight.reweight("ee_mumu", p, w, synth.ORIG_EW, [synth.NEW_EE])
    assert rel_err(got, ref).max() < 1e-12
    # an event generated with alpha_s = 0 has |M|^2 = 0: w' = 0
    q = synth.events("uu_eeg", n)
    a = np.full(n, 0.118)
    a[3] = 0.0
    got = _run("uu_eeg", q, np.ones(n), synth.ORIG_EW, [synth.NEW_UU], a, np.full(n, 91.1876))
    assert got[0, 3] == 0.0 and np.all(got[0, np.arange(n) != 3] > 0)
