"""rwgt_eval and rwgt_me2 with arrays in host memory.

The library tells device from host memory with hipPointerGetAttributes and
copies host arrays through a device staging buffer, so the device work is the
same as for device arrays: results must be equal bit for bit, for every
placement of momenta, input weights and output (device, pinned host, pageable
host), in FP64 and in the mixed mode.  With a pageable array the call waits
for its stream, so the output is read here without synchronising first; with
pinned arrays only it stays asynchronous and the test synchronises.  One case
per process is also held against the oracle (tolerances as the parity tests:
1e-11 for u u~ -> e+ e- g, 1e-10 for g g -> t t~ g g |M|^2).
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import reweight

from gpu_util import PROCESS_TEXT, rel_err, torch_cuda

pytestmark = pytest.mark.gpu

PLACES = ("device", "pinned", "pageable")


def _case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _place(torch, x, where):
    t = torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64))
    if where == "device":
        return t.cuda()
    if where == "pinned":
        return t.pin_memory()
    return t.clone()


def _empty(torch, shape, where):
    if where == "device":
        return torch.full(shape, -1.0, dtype=torch.float64, device="cuda")
    t = torch.full(shape, -1.0, dtype=torch.float64)
    return t.pin_memory() if where == "pinned" else t


def _read(torch, t, places):
    if "pageable" not in places:
        torch.cuda.synchronize()
    return t.cpu().numpy() if t.is_cuda else t.numpy().copy()


@pytest.mark.parametrize("precision", [0, 1])
def test_eval_every_placement(precision):
    import paper_2510_05100_amd as rw
    torch = torch_cuda()
    n = 3000                                      # several tiles and a ragged tail
    _case("host_eval_placements", process="uu_eeg", n=n, precision=precision)
    p = synth.events("uu_eeg", n, seed=71)
    w = np.linspace(0.5, 1.5, n)
    cards = [synth.NEW_UU, synth.NEW_EE]
    rows = np.stack([c.row("uu_eeg") for c in cards])
    with rw.Reweighter(PROCESS_TEXT["uu_eeg"], synth.ORIG_EW.slha(), precision) as r:
        ref = _empty(torch, (2, n), "device")
        r.eval(_place(torch, p, "device"), _place(torch, w, "device"), rows, ref)
        torch.cuda.synchronize()
        ref = ref.cpu().numpy()
        for wp, ww, wo in itertools.product(PLACES, PLACES, PLACES):
            out = _empty(torch, (2, n), wo)
            r.eval(_place(torch, p, wp), _place(torch, w, ww), rows, out)
            got = _read(torch, out, (wp, ww, wo))
            assert np.array_equal(got, ref), (wp, ww, wo)
    if precision == 0:
        want, _, _ = reweight.reweight("uu_eeg", p, w, synth.ORIG_EW, cards)
        assert rel_err(ref, want).max() < 1e-11


def test_me2_host_gg_ttgg():
    import paper_2510_05100_amd as rw
    torch = torch_cuda()
    n = 300
    _case("host_me2", process="gg_ttgg", n=n)
    p = synth.events("gg_ttgg", n, seed=72)
    rows = np.stack([c.row("gg_ttgg") for c in (synth.ORIG_QCD, synth.NEW_QCD)])
    with rw.Reweighter(PROCESS_TEXT["gg_ttgg"], synth.ORIG_QCD.slha(), 0) as r:
        ref = _empty(torch, (2, n), "device")
        r.me2(_place(torch, p, "device"), rows, ref)
        torch.cuda.synchronize()
        ref = ref.cpu().numpy()
        for wp, wo in [("pageable", "pageable"), ("pinned", "pinned"), ("device", "pageable"), ("pinned", "device")]:
            out = _empty(torch, (2, n), wo)
            r.me2(_place(torch, p, wp), rows, out)
            assert np.array_equal(_read(torch, out, (wp, wo)), ref), (wp, wo)
    for k, c in enumerate((synth.ORIG_QCD, synth.NEW_QCD)):
        assert rel_err(ref[k], reweight.me2("gg_ttgg", p, c)).max() < 1e-10


def test_staging_grows_and_shrinks():
    """Calls of 3000, 9000, 100 and 0 events on one context, host arrays each
    time: the staging buffer is regrown once and reused; every call equals
    the device path."""
    import paper_2510_05100_amd as rw
    torch = torch_cuda()
    p_all = synth.events("uu_eeg", 9000, seed=73)
    rows = synth.NEW_UU.row("uu_eeg")[None, :]
    with rw.Reweighter(PROCESS_TEXT["uu_eeg"], synth.ORIG_EW.slha(), 0) as r:
        for n in (3000, 9000, 100, 0):
            _case("host_staging", n=n)
            p = p_all[:n]
            w = np.ones(n)
            ref = _empty(torch, (1, n), "device")
            r.eval(_place(torch, p, "device"), _place(torch, w, "device"), rows, ref)
            out = _empty(torch, (1, n), "pinned")
            r.eval(_place(torch, p, "pinned"), _place(torch, w, "pageable"), rows, out)
            torch.cuda.synchronize()
            assert np.array_equal(out.numpy(), ref.cpu().numpy())


def test_nonfinite_with_host_output():
    """The non-finite count reads the staged output: one event with a NaN
    momentum gives NaN weights for both cards and a count of 2."""
    import paper_2510_05100_amd as rw
    torch = torch_cuda()
    n = 500
    _case("host_nonfinite", n=n)
    p = synth.events("uu_eeg", n, seed=74)
    p[123, 2, 1] = np.nan
    rows = np.stack([c.row("uu_eeg") for c in (synth.NEW_UU, synth.NEW_EE)])
    with rw.Reweighter(PROCESS_TEXT["uu_eeg"], synth.ORIG_EW.slha(), 0) as r:
        out = _empty(torch, (2, n), "pageable")
        r.eval(_place(torch, p, "pageable"), _place(torch, np.ones(n), "pageable"), rows, out)
        got = out.numpy()
        assert rw.rwgt_nonfinite(r.ctx) == 2
        assert np.isnan(got[:, 123]).all() and np.isfinite(np.delete(got, 123, axis=1)).all()
