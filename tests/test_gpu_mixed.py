"""Mixed precision (float amplitudes; FP16 hi/lo or BF16 hi/mid/lo matrix-core
colour sum for g g -> t t~ g g; FP64 momenta, denominators and ratio) against
the FP64 oracle.

Tolerances: the reweighting target is a maximum relative error of 1e-5 on w'
against the oracle.  |M|^2 itself carries the float rounding of the
amplitudes amplified by the cancellation between diagrams (the paper warns of
it for single precision); it is checked at 1e-4 relative, which bounds an
amplification of ~1e3 over float epsilon.
"""
import numpy as np
import pytest

import synth
from oracle import reweight

from gpu_util import gpu_eval, gpu_me2, rel_err

pytestmark = pytest.mark.gpu

RATIO = (0.130 / 0.118) ** 4
MIXED = {"fp16": 1, "bf16": 2}


@pytest.mark.parametrize("mode", ["fp16", "bf16"])
def test_gg_ttgg_mixed(mode):
    n = 300
    print(f"[case] gg_ttgg_mixed mode={mode} n={n}", flush=True)
    p = synth.events("gg_ttgg", n)
    me = gpu_me2("gg_ttgg", p, synth.ORIG_QCD, [synth.ORIG_QCD], MIXED[mode])[0]
    ref = reweight.me2("gg_ttgg", p, synth.ORIG_QCD)
    err = rel_err(me, ref)
    print(f"gg_ttgg {mode} |M|^2 max rel err {err.max():.3g} median {np.median(err):.3g}", flush=True)
    assert err.max() < 1e-4
    w = gpu_eval("gg_ttgg", p, np.ones(n), synth.ORIG_QCD, [synth.NEW_QCD], MIXED[mode])[0]
    werr = np.abs(w / RATIO - 1)
    print(f"gg_ttgg {mode} w' max rel err {werr.max():.3g}", flush=True)
    assert werr.max() < 1e-5


@pytest.mark.parametrize("process,orig,new,n", [
    ("ee_mumu", synth.ORIG_EW, synth.NEW_EE, 3000),
    ("uu_eeg", synth.ORIG_EW, synth.NEW_UU, 2000),
])
def test_electroweak_mixed(process, orig, new, n):
    print(f"[case] {process}_mixed n={n}", flush=True)
    p = synth.events(process, n)
    me = gpu_me2(process, p, orig, [orig, new], MIXED["fp16"])
    for k, c in enumerate([orig, new]):
        assert rel_err(me[k], reweight.me2(process, p, c)).max() < 1e-4
    w = gpu_eval(process, p, np.ones(n), orig, [new], MIXED["fp16"])
    ref, _, _ = reweight.reweight(process, p, np.ones(n), orig, [new])
    err = rel_err(w, ref)
    print(f"{process} mixed w' max rel err {err.max():.3g}", flush=True)
    assert err.max() < 1e-5


def test_mixed_ragged_last_wave():
    # 64-lane waves cooperate in the matrix-core colour sum: event counts that
    # end inside a wave must still give every event its own result
    for n in (1, 65, 130):
        print(f"[case] mixed ragged n={n}", flush=True)
        p = synth.events("gg_ttgg", n)
        me = gpu_me2("gg_ttgg", p, synth.ORIG_QCD, [synth.ORIG_QCD], MIXED["fp16"])[0]
        ref = reweight.me2("gg_ttgg", p, synth.ORIG_QCD)
        assert rel_err(me, ref).max() < 1e-4


def test_fp64_ragged_last_workgroup():
    # the two waves of a workgroup split each event's helicity sum and add
    # through LDS: a last workgroup with fewer than 64 events (lanes past the
    # end recompute the last event and write nothing)
    for n in (1, 65, 127):
        print(f"[case] fp64 ragged n={n}", flush=True)
        p = synth.events("gg_ttgg", n)
        me = gpu_me2("gg_ttgg", p, synth.ORIG_QCD, [synth.ORIG_QCD, synth.NEW_QCD])
        ref = reweight.me2("gg_ttgg", p, synth.ORIG_QCD)
        assert rel_err(me[0], ref).max() < 1e-10
        assert np.max(np.abs(me[1] / me[0] / ((0.130 / 0.118) ** 4) - 1)) < 1e-12
