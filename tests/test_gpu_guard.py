"""The mixed path's cancellation guard (rwgt_set_mixed_guard).

For each event the mixed kernel measures kappa, the ratio of the incoherent
to the coherent sum of the amplitude terms over flows and helicities (largest
over the cards); events with kappa above the threshold are evaluated again in
double precision within the same call.  Contract, checked event by event on
20,000 events of each process with a threshold of 30 (a few percent flagged,
so that both sets are large):
- the events re-evaluated are exactly those with kappa above the threshold
  (kappa from rwgt_cancellation, the same kernel without re-evaluation), and
  rwgt_mixed_guard_count reports their number;
- their w' equals the double-precision path's to 4e-15 (the same generated
  code, evaluated one lane per helicity instead of one lane per event, so
  the compiler may round a last bit differently), the others' equals the
  unguarded mixed path's bit for bit;
- kappa is positive and finite.
"""
import numpy as np
import pytest

import synth

from gpu_util import PROCESS_TEXT, dev, torch_cuda

pytestmark = pytest.mark.gpu

CASES = [("gg_ttgg", synth.ORIG_QCD, synth.NEW_QCD, 1), ("gg_ttgg", synth.ORIG_QCD, synth.NEW_QCD, 2),
         ("uu_eeg", synth.ORIG_EW, synth.NEW_UU, 1), ("ee_mumu", synth.ORIG_EW, synth.NEW_EE, 1)]


def _eval(rw, torch, process, orig, new, precision, p, w, guard=None):
    ctx = rw.rwgt_create(PROCESS_TEXT[process], orig.slha(), precision)
    try:
        rw.rwgt_set_stream(ctx, None)
        if guard is not None:
            rw.rwgt_set_mixed_guard(ctx, guard)
        out = torch.empty((1, p.shape[0]), dtype=torch.float64, device="cuda")
        rw.rwgt_eval(ctx, p, w, new.row(process), out)
        n = rw.rwgt_mixed_guard_count(ctx)
        kappa = None
        if precision != 0:
            kappa = torch.empty(p.shape[0], dtype=torch.float64, device="cuda")
            rw.rwgt_cancellation(ctx, p, np.stack([orig.row(process), new.row(process)]), kappa)
            kappa = kappa.cpu().numpy()
        torch.cuda.synchronize()
        return out.cpu().numpy()[0], n, kappa
    finally:
        rw.rwgt_destroy(ctx)


@pytest.mark.parametrize("process,orig,new,precision", CASES)
def test_guard_contract(process, orig, new, precision):
    n = 20_000
    print(f"[case] guard {process} precision={precision} n={n}", flush=True)
    torch = torch_cuda()
    import paper_2510_05100_amd as rw
    p = dev(synth.events(process, n))
    w = dev(np.linspace(0.5, 2.0, n))
    w64, n64, _ = _eval(rw, torch, process, orig, new, 0, p, w)
    plain, n_off, kappa = _eval(rw, torch, process, orig, new, precision, p, w, guard=0.0)
    guarded, n_on, kappa2 = _eval(rw, torch, process, orig, new, precision, p, w, guard=30.0)
    assert n64 == 0 and n_off == 0
    np.testing.assert_array_equal(kappa, kappa2)
    assert np.all(np.isfinite(kappa)) and np.all(kappa > 0)
    flagged = kappa > 30.0
    print(f"{process}: {flagged.sum()} of {n} flagged (kappa median {np.median(kappa):.3g}, max {kappa.max():.3g})",
          flush=True)
    assert n_on == int(flagged.sum())
    # re-evaluated events: FP64, from a one-wave-per-event kernel (a lane per helicity) whose
    # instruction selection may round a last bit differently from the FP64 path's kernel
    assert np.max(np.abs(guarded[flagged] / w64[flagged] - 1.0), initial=0.0) <= 4e-15
    np.testing.assert_array_equal(guarded[~flagged], plain[~flagged])
    if process == "ee_mumu":
        assert n_on == 0                       # two diagrams (photon, Z) that barely cancel at 200 GeV: kappa <= 4
    else:
        assert 0 < n_on < 0.2 * n


def test_guard_rejects_nan_threshold():
    print("[case] guard arguments", flush=True)
    torch_cuda()
    import paper_2510_05100_amd as rw
    ctx = rw.rwgt_create(PROCESS_TEXT["gg_ttgg"], synth.ORIG_QCD.slha(), 0)
    try:
        with pytest.raises(rw.RwgtError, match="EINVAL"):
            rw.rwgt_set_mixed_guard(ctx, float("nan"))
        kappa = dev(np.zeros(4))
        with pytest.raises(rw.RwgtError, match="mixed path"):
            rw.rwgt_cancellation(ctx, dev(synth.events("gg_ttgg", 4)), synth.ORIG_QCD.row("gg_ttgg"), kappa)
    finally:
        rw.rwgt_destroy(ctx)
