"""Batched persistent launch against the plain path and the oracle.

Each segment's w' must equal what rwgt_eval gives for the same events and
card: the same generated arithmetic runs in both kernels, so the results agree
to a few ulp (1e-14 relative is the bar; the compiler may contract the two
kernels' expressions differently).  Sampled events are also checked against
the oracle at the FP64 parity bars (1e-12 / 1e-11).
"""
import os

import numpy as np
import pytest

import synth
from oracle import reweight

from gpu_util import PROCESS_TEXT, dev, rel_err, torch_cuda

pytestmark = pytest.mark.gpu


def _setup(precision=0, ncards=6, seed=7):
    torch = torch_cuda()
    import paper_2510_05100_amd as rw
    grid = synth.batch_grid()
    rng = np.random.default_rng(seed)
    cards = [grid[i] for i in rng.choice(64, ncards, replace=False)]
    counts = rng.integers(50, 1500, size=(ncards, 2))
    counts[0, 1] = 1                       # one-event segment
    counts[1, 0] = 0                       # empty segment
    pools = {"ee_mumu": synth.events("ee_mumu", 1500), "uu_eeg": synth.events("uu_eeg", 1500)}
    dpools = {k: dev(v) for k, v in pools.items()}
    ctxs = [rw.rwgt_create(PROCESS_TEXT["ee_mumu"], synth.ORIG_EW.slha(), precision),
            rw.rwgt_create(PROCESS_TEXT["uu_eeg"], synth.ORIG_EW.slha(), precision)]
    jobs = []
    for c, card in enumerate(cards):
        for j, proc in enumerate(("ee_mumu", "uu_eeg")):
            n = int(counts[c, j])
            w = np.linspace(0.5, 1.5, max(n, 1))[:n]
            jobs.append(dict(ctx=j, proc=proc, n=n, card=card, w=w, w_dev=dev(w),
                             mom=dpools[proc][:n].contiguous(),
                             out=torch.full((n,), -1.0, dtype=torch.float64, device="cuda")))
    return torch, rw, ctxs, jobs, pools


def _segments(rw, jobs):
    return rw.make_segments((j["ctx"], j["mom"], j["w_dev"], j["card"].row(j["proc"]), j["out"]) for j in jobs)


def _plain(torch, rw, ctxs, job):
    out = torch.empty((1, job["n"]), dtype=torch.float64, device="cuda")
    rw.rwgt_set_stream(ctxs[job["ctx"]], None)
    rw.rwgt_eval(ctxs[job["ctx"]], job["mom"], job["w_dev"], job["card"].row(job["proc"]), out)
    return out


@pytest.mark.parametrize("hel_split", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_batch_matches_plain_and_oracle(precision, hel_split):
    """Both batch kernels (one lane per event; one lane per (event, card,
    helicity), tiles of 96 events so that groups end inside tiles and
    segments) equal the plain path to the bit."""
    print(f"[case] batch precision={precision} hel_split={hel_split}", flush=True)
    torch, rw, ctxs, jobs, pools = _setup(precision)
    for c in ctxs:                             # the batched form has no cancellation guard: compare unguarded
        rw.rwgt_set_mixed_guard(c, 0.0)
    b = rw.rwgt_batch_create(ctxs)
    try:
        segs, keep = _segments(rw, jobs)
        if hel_split:
            rw.rwgt_batch_set_schedule(b, 96, 256, 2, 1)
            assert rw.rwgt_batch_get_schedule(b)["hel_split"] == 1
        rw.rwgt_batch_eval(b, segs)
        torch.cuda.synchronize()
        for job in jobs:
            if job["n"] == 0:
                continue
            ref = _plain(torch, rw, ctxs, job)
            torch.cuda.synchronize()
            got = job["out"].cpu().numpy()
            assert np.array_equal(got, ref.cpu().numpy()[0])
        # sampled events against the oracle: FP64 at the parity bars, mixed at 1e-5 (w' target)
        for job in jobs[:4]:
            if job["n"] == 0:
                continue
            idx = np.arange(0, job["n"], max(1, job["n"] // 40))
            want, _, _ = reweight.reweight(job["proc"], pools[job["proc"]][idx], job["w"][idx],
                                           synth.ORIG_EW, [job["card"]])
            bar = 1e-5 if precision else (1e-12 if job["proc"] == "ee_mumu" else 1e-11)
            assert np.max(rel_err(job["out"].cpu().numpy()[idx], want[0])) < bar
    finally:
        rw.rwgt_batch_destroy(b)
        for c in ctxs:
            rw.rwgt_destroy(c)


def test_graph_replay_sees_new_inputs_and_recaptures():
    print("[case] batch replay", flush=True)
    torch, rw, ctxs, jobs, _ = _setup(0, ncards=4, seed=3)
    b = rw.rwgt_batch_create(ctxs)
    try:
        segs, keep = _segments(rw, jobs)
        rw.rwgt_batch_eval(b, segs)
        torch.cuda.synchronize()
        first = [j["out"].clone() for j in jobs]
        for j in jobs:                         # same shapes, new weights: the graph is replayed
            j["w_dev"].mul_(3.0)
        rw.rwgt_batch_eval(b, segs)
        torch.cuda.synchronize()
        for j, f in zip(jobs, first):
            if j["n"]:
                np.testing.assert_allclose(j["out"].cpu().numpy(), 3.0 * f.cpu().numpy(), rtol=1e-15)
        # several replays in a row, with eager work and synchronisations between
        # them (outputs cleared, weights rescaled): every replay resets its tile
        # counter inside the graph and writes every output again
        scale = 3.0
        for rep in range(5):
            for j in jobs:
                j["out"].fill_(-1.0)
                j["w_dev"].mul_(0.5)
            scale *= 0.5
            torch.cuda.synchronize()
            rw.rwgt_batch_eval(b, segs)
            torch.cuda.synchronize()
            for j, f in zip(jobs, first):
                if j["n"]:
                    np.testing.assert_allclose(j["out"].cpu().numpy(), scale * f.cpu().numpy(), rtol=1e-15,
                                               err_msg=f"replay {rep}")
        for j in jobs:
            j["w_dev"].mul_(3.0 / scale)
        # a different schedule changes the launch shape: captured again, same results
        rw.rwgt_batch_set_schedule(b, 64, 64, 1)
        for j in jobs:
            j["out"].fill_(-1.0)
        rw.rwgt_batch_eval(b, segs)
        torch.cuda.synchronize()
        for j, f in zip(jobs, first):
            if j["n"]:
                np.testing.assert_allclose(j["out"].cpu().numpy(), 3.0 * f.cpu().numpy(), rtol=1e-15)
        # fewer segments: captured again
        rw.rwgt_batch_eval(b, segs[:3])
        torch.cuda.synchronize()
        assert rw.rwgt_batch_time(b) >= 0.0
    finally:
        rw.rwgt_batch_destroy(b)
        for c in ctxs:
            rw.rwgt_destroy(c)


def test_tune_picks_a_schedule(tmp_path):
    print("[case] batch tune", flush=True)
    os.environ["RWGT_TUNE_CACHE"] = str(tmp_path / "tune.txt")
    torch, rw, ctxs, jobs, _ = _setup(0, ncards=3, seed=5)
    b = rw.rwgt_batch_create(ctxs)
    try:
        segs, keep = _segments(rw, jobs)
        sched = rw.rwgt_batch_tune(b, segs, reps=1)
        assert sched["tile_events"] >= 64 and sched["block"] in (64, 128, 256) and sched["grid"] >= 1
        assert sched["hel_split"] in (0, 1)
        text = (tmp_path / "tune.txt").read_text()
        assert "gfx950" in text and "|" in text
        rw.rwgt_batch_eval(b, segs)
        torch.cuda.synchronize()
        for job in jobs:
            if job["n"]:
                ref = _plain(torch, rw, ctxs, job)
                torch.cuda.synchronize()
                assert np.max(rel_err(job["out"].cpu().numpy(), ref.cpu().numpy()[0])) < 1e-14
    finally:
        os.environ.pop("RWGT_TUNE_CACHE", None)
        rw.rwgt_batch_destroy(b)
        for c in ctxs:
            rw.rwgt_destroy(c)


def test_batch_rejects_bad_segments():
    print("[case] batch errors", flush=True)
    torch, rw, ctxs, jobs, _ = _setup(0, ncards=2, seed=9)
    b = rw.rwgt_batch_create(ctxs)
    try:
        segs, keep = _segments(rw, jobs)
        segs[0].ctx = 5
        with pytest.raises(rw.RwgtError, match="EINVAL"):
            rw.rwgt_batch_eval(b, segs)
    finally:
        rw.rwgt_batch_destroy(b)
        for c in ctxs:
            rw.rwgt_destroy(c)
    gg = rw.rwgt_create(PROCESS_TEXT["gg_ttgg"], synth.ORIG_QCD.slha())
    try:
        with pytest.raises(rw.RwgtError, match="EPROCESS"):
            rw.rwgt_batch_create([gg])
    finally:
        rw.rwgt_destroy(gg)
