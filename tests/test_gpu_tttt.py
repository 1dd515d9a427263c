"""g g -> t t~ t t~ (pure QCD) through the C ABI against the colour-dressed
oracle (oracle/qcd_dressed.py).

Tolerances:
- FP64: the device path (diagrams with HELAS-style currents, colour flows in a
  Fierz-reduced basis of two generator strings) and the oracle (recursion
  over subsets of legs with every colour index open) evaluate |M|^2 in double
  with different algorithms, 1e-10 relative as for g g -> t t~ g g.  The
  alpha_s-only card gives w'/w = (0.130/0.118)^4 exactly, to 1e-12 on every
  event.
- Mixed precision (float amplitudes, FP16 colour sum on the matrix cores, the
  cancellation guard on): 1e-5 relative against the oracle on sampled events
  and on the ratio over every event.
Sampled events include the first, the last (a ragged tail of the 128-lane
workgroups) and spread indices; 203 events span four workgroups.
"""
import functools

import numpy as np
import pytest

import synth
from oracle import reweight

from gpu_util import dev, gpu_eval, gpu_me2, rel_err, torch_cuda

pytestmark = pytest.mark.gpu

RATIO = (0.130 / 0.118) ** 4
N = 203
SAMPLE = [0, 1, 64, 127, 150, N - 1]


def _case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


@functools.lru_cache(maxsize=None)
def _events():
    return synth.events("gg_tttt", N)


@functools.lru_cache(maxsize=None)
def _oracle_me2():
    return reweight.me2("gg_tttt", _events()[SAMPLE], synth.ORIG_QCD)


def test_fp64_me2_against_oracle():
    _case("gg_tttt_fp64", n=N)
    p = _events()
    me = gpu_me2("gg_tttt", p, synth.ORIG_QCD, [synth.ORIG_QCD, synth.NEW_QCD])
    assert np.all(np.isfinite(me)) and np.all(me > 0)
    assert rel_err(me[0][SAMPLE], _oracle_me2()).max() < 1e-10
    assert rel_err(me[1] / me[0], np.full(N, RATIO)).max() < 1e-12


def test_fp64_reweighting_ratio_every_event():
    n = 5000
    _case("gg_tttt_fp64_ratio", n=n)
    p = synth.events("gg_tttt", n, seed=71)
    w = np.linspace(0.5, 1.5, n)
    wn = gpu_eval("gg_tttt", p, w, synth.ORIG_QCD, [synth.NEW_QCD])
    assert rel_err(wn[0], w * RATIO).max() < 1e-12


@pytest.mark.parametrize("precision", [1, 2])
def test_mixed_against_oracle(precision):
    _case("gg_tttt_mixed", n=N, precision=precision)
    p = _events()
    me = gpu_me2("gg_tttt", p, synth.ORIG_QCD, [synth.ORIG_QCD], precision=precision)[0]
    assert rel_err(me[SAMPLE], _oracle_me2()).max() < 1e-5
    w = np.ones(N)
    wn = gpu_eval("gg_tttt", p, w, synth.ORIG_QCD, [synth.NEW_QCD], precision=precision)[0]
    assert rel_err(wn, np.full(N, RATIO)).max() < 1e-5


def test_factored_and_running_alphas():
    """The coupling-factored path (one evaluation, |M|^2 scales as alpha_s^4)
    and the per-event running alpha_s path agree with the full path."""
    import paper_2510_05100_amd as rw
    torch = torch_cuda()
    n = 1000
    _case("gg_tttt_factored_alphas", n=n)
    p = synth.events("gg_tttt", n, seed=72)
    w = np.linspace(0.5, 1.5, n)
    rows = synth.NEW_QCD.row("gg_tttt")[None, :]
    with rw.Reweighter("g g > t t~ t t~", synth.ORIG_QCD.slha()) as r:
        full = torch.empty((1, n), dtype=torch.float64, device="cuda")
        fac = torch.empty_like(full)
        run = torch.empty_like(full)
        r.eval(dev(p), dev(w), rows, full)
        r.eval_factored(dev(p), dev(w), rows, fac)
        scales = np.full(n, 91.1876)                      # at the reference scale running changes nothing
        rw.rwgt_eval_alphas(r.ctx, dev(p), dev(w), None, dev(scales), rows, run)
        torch.cuda.synchronize()
        f, fc, rn = full.cpu().numpy(), fac.cpu().numpy(), run.cpu().numpy()
    assert rel_err(fc, f).max() < 1e-12
    assert rel_err(rn, f).max() < 1e-12


def test_full_size_workload():
    """The bench's four-top workload: 1e6 events, alpha_s 0.118 -> 0.130.
    FP64: w'/w exact on every event (1e-12) and |M|^2 against the oracle on
    four spread events (1e-10); mixed with the guard: w' within 1e-5 of the
    exact ratio on every event and |M|^2 within 1e-5 on the samples; no
    non-finite output."""
    import paper_2510_05100_amd as rw
    torch = torch_cuda()
    n = 1_000_000
    _case("gg_tttt_full", n=n)
    p = synth.events("gg_tttt", n)
    idx = np.array([0, 333_333, 777_777, n - 1])
    ref = reweight.me2("gg_tttt", p[idx], synth.ORIG_QCD)
    pd, wd = dev(p), dev(np.ones(n))
    rows = synth.NEW_QCD.row("gg_tttt")[None, :]
    for prec, bar_w, bar_me in ((0, 1e-12, 1e-10), (1, 1e-5, 1e-5)):
        with rw.Reweighter("g g > t t~ t t~", synth.ORIG_QCD.slha(), prec) as r:
            out = torch.empty((1, n), dtype=torch.float64, device="cuda")
            r.eval(pd, wd, rows, out)
            assert rw.rwgt_nonfinite(r.ctx) == 0
            me = torch.empty((1, n), dtype=torch.float64, device="cuda")
            r.me2(pd, synth.ORIG_QCD.row("gg_tttt"), me)
            torch.cuda.synchronize()
            wn, mh = out.cpu().numpy()[0], me.cpu().numpy()[0]
        assert rel_err(wn, np.full(n, RATIO)).max() < bar_w, prec
        assert rel_err(mh[idx], ref).max() < bar_me, prec


def test_flop_counts_with_helicity_reversal():
    """The pure-QCD processes evaluate one helicity of each reversed pair:
    the executed count is half the plain sum over the 64 kept helicities (up
    to the final averaging multiply); the electroweak processes evaluate every
    kept helicity."""
    import paper_2510_05100_amd as rw
    from gpu_util import PROCESS_TEXT
    torch_cuda()
    for name, card, halved in (("gg_ttgg", synth.ORIG_QCD, True), ("gg_tttt", synth.ORIG_QCD, True),
                               ("uu_eeg", synth.ORIG_EW, False), ("ee_mumu", synth.ORIG_EW, False)):
        _case("flops", process=name)
        with rw.Reweighter(PROCESS_TEXT[name], card.slha()) as r:
            full, run = rw.rwgt_flops(r.ctx), rw.rwgt_flops_executed(r.ctx)
            info = rw.rwgt_process_info(r.ctx)
        assert full > 0 and run > 0
        if halved:
            assert info["nhel_kept"] == 64
            assert abs((full - 1.0) / (run - 1.0) - 2.0) < 1e-12, (name, full, run)
        else:
            assert run == full, name


@pytest.mark.parametrize("n", [1, 65, 127])
def test_fp64_ragged_workgroups(n):
    """A single event and partly filled last workgroups (64 events per
    128-lane workgroup): the first and last events against the oracle."""
    _case("gg_tttt_ragged", n=n)
    p = synth.events("gg_tttt", n, seed=75)
    idx = sorted({0, n - 1})
    me = gpu_me2("gg_tttt", p, synth.ORIG_QCD, [synth.ORIG_QCD])[0]
    assert np.all(np.isfinite(me)) and np.all(me > 0)
    assert rel_err(me[idx], reweight.me2("gg_tttt", p[idx], synth.ORIG_QCD)).max() < 1e-10


def test_several_cards_in_one_call():
    """Five cards in one call (the two waves of each workgroup add their
    helicity halves through LDS once per card): w'/w = (alpha_s'/0.118)^4
    on every event for every card, the original card giving 1."""
    import dataclasses
    n = 300
    _case("gg_tttt_cards", n=n)
    p = synth.events("gg_tttt", n, seed=76)
    alphas = (0.100, 0.118, 0.125, 0.130, 0.140)
    cards = [dataclasses.replace(synth.ORIG_QCD, aS=a) for a in alphas]
    w = np.linspace(0.5, 2.0, n)
    wn = gpu_eval("gg_tttt", p, w, synth.ORIG_QCD, cards)
    for k, a in enumerate(alphas):
        assert np.max(np.abs(wn[k] / w / ((a / 0.118) ** 4) - 1)) < 1e-12, a
