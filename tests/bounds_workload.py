"""Child process of tests/test_gpu_bounds_check.py: drives every checked
device kernel of the bounds-checked library (RWGT_LIBRARY=check) with ragged
sizes and reports, after each step, the indices found out of range.

Steps: the gg -> tt~gg kernels (FP64 with two new cards, the FP16 and BF16
guarded mixed kernels and their FP64 re-evaluation, |M|^2 only, kappa),
gg -> tt~tt~, u u~ -> e+ e- g and e+ e- -> mu+ mu- in both precisions, the
cross sections, the factored and running-alpha_s paths, the batched kernels
in both schedules, the card-per-event kernel (with out-of-range card
indices, which it must reject before reading), host arrays through the
staging buffer.  Prints "step <name> misses <n>" per step and exits 1 if any
step saw one; the FP64 gg -> tt~gg |M|^2 is also held against the oracle.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from gpu_util import PROCESS_TEXT, dev, rel_err, torch_cuda  # noqa: E402
from oracle import reweight  # noqa: E402


def main():
    assert os.environ.get("RWGT_LIBRARY") == "check"
    torch = torch_cuda()
    import paper_2510_05100_amd as rw
    enabled, _ = rw.rwgt_bounds_check()
    print(f"library {rw._abi.LIB_PATH} checked={enabled}", flush=True)
    if not enabled:
        return 2
    bad = []

    def step(name):
        torch.cuda.synchronize()
        _, n = rw.rwgt_bounds_check()
        print(f"step {name} misses {n}", flush=True)
        if n:
            bad.append(name)

    def out(shape):
        return torch.full(shape, -1.0, dtype=torch.float64, device="cuda")

    # g g -> t t~ g g: 203 events (a ragged last workgroup), two new cards
    n = 203
    p = synth.events("gg_ttgg", n)
    pd, wd = dev(p), dev(np.linspace(0.5, 1.5, n))
    cards = np.stack([synth.NEW_QCD.row("gg_ttgg"), synth.ORIG_QCD.row("gg_ttgg")])
    for prec in (0, 1, 2):
        with rw.Reweighter(PROCESS_TEXT["gg_ttgg"], synth.ORIG_QCD.slha(), prec) as r:
            if prec:
                rw.rwgt_set_mixed_guard(r.ctx, 1.0)          # flag many events: the re-evaluation kernel runs
            w = out((2, n))
            r.eval(pd, wd, cards, w)
            me = out((1, n))
            r.me2(pd, synth.ORIG_QCD.row("gg_ttgg"), me)
            if prec:
                kappa = out((n,))
                rw.rwgt_cancellation(r.ctx, pd, cards, kappa)
            step(f"gg_ttgg precision {prec}")
            if prec == 0:
                idx = [0, 101, n - 1]
                err = rel_err(me.cpu().numpy()[0][idx], reweight.me2("gg_ttgg", p[idx], synth.ORIG_QCD)).max()
                print(f"gg_ttgg |M|^2 against the oracle: {err:.2e}", flush=True)
                if not err < 1e-10:
                    bad.append("gg_ttgg parity")
            rw.rwgt_eval_factored(r.ctx, pd, wd, cards, out((2, n)))
            step(f"gg_ttgg factored precision {prec}")
            rw.rwgt_eval_alphas(r.ctx, pd, wd, None, dev(np.linspace(50.0, 900.0, n)), cards, out((2, n)))
            step(f"gg_ttgg running alpha_s precision {prec}")

    # g g -> t t~ t t~
    n = 130
    p4 = dev(synth.events("gg_tttt", n))
    for prec in (0, 1):
        with rw.Reweighter(PROCESS_TEXT["gg_tttt"], synth.ORIG_QCD.slha(), prec) as r:
            r.eval(p4, dev(np.ones(n)), synth.NEW_QCD.row("gg_tttt")[None, :], out((1, n)))
            step(f"gg_tttt precision {prec}")

    # electroweak processes, cross sections, factored, host arrays
    for proc, n in (("uu_eeg", 3001), ("ee_mumu", 777)):
        pe = synth.events(proc, n)
        pd, wd = dev(pe), dev(np.linspace(0.5, 1.5, n))
        rows = np.stack([c.row(proc) for c in synth.batch_grid()[:3]])
        for prec in (0, 1):
            with rw.Reweighter(PROCESS_TEXT[proc], synth.ORIG_EW.slha(), prec) as r:
                w = out((3, n))
                r.eval(pd, wd, rows, w)
                rw.rwgt_xsec(r.ctx, wd, w, 10.0, 0.1, 10.0 / n)
                rw.rwgt_xsec(r.ctx, wd, w, 10.0, 0.1, 10.0 / n, entry="rwgt_xsec_noalloc")
                rw.rwgt_eval_factored(r.ctx, pd, wd, rows, out((3, n)))
                host = torch.full((3, n), -1.0, dtype=torch.float64).pin_memory()
                r.eval(torch.as_tensor(pe).pin_memory(), torch.as_tensor(np.ones(n)), rows, host)
                step(f"{proc} precision {prec}")

    # batched kernels: segments of both processes, one empty and one single-event segment
    grid = synth.batch_grid()
    pools = {k: dev(synth.events(k, 700)) for k in ("ee_mumu", "uu_eeg")}
    for prec in (0, 1):
        ctxs = [rw.rwgt_create(PROCESS_TEXT["ee_mumu"], synth.ORIG_EW.slha(), prec),
                rw.rwgt_create(PROCESS_TEXT["uu_eeg"], synth.ORIG_EW.slha(), prec)]
        b = rw.rwgt_batch_create(ctxs)
        try:
            keep, jobs = [], []
            for s, (j, nseg) in enumerate([(0, 300), (1, 0), (1, 1), (0, 699), (1, 513)]):
                proc = ("ee_mumu", "uu_eeg")[j]
                w = dev(np.ones(max(nseg, 1)))[:nseg]
                o = out((nseg,))
                keep += [w, o]
                jobs.append((j, pools[proc][:nseg].contiguous(), w, grid[s].row(proc), o))
            segs, k2 = rw.make_segments(jobs)
            for hel_split in (0, 1):
                rw.rwgt_batch_set_schedule(b, 96, 256, 2, hel_split)
                rw.rwgt_batch_eval(b, segs)
                step(f"batch precision {prec} hel_split {hel_split}")
        finally:
            rw.rwgt_batch_destroy(b)
            for c in ctxs:
                rw.rwgt_destroy(c)

    # card-per-event kernel, with indices outside the table
    n = 999
    pu = dev(synth.events("uu_eeg", n))
    table = np.stack([c.row("uu_eeg") for c in grid[:8]])
    cidx = (np.arange(n) % 8).astype(np.int32)
    cidx[[5, 500, 998]] = [-1, 8, 1 << 30]
    with rw.Reweighter(PROCESS_TEXT["uu_eeg"], synth.ORIG_EW.slha(), 0) as r:
        rw.rwgt_eval_cards(r.ctx, pu, dev(np.ones(n)), table, torch.as_tensor(cidx).cuda(), out((n,)))
        step("card per event")

    print("bounds check failed in: " + ", ".join(bad) if bad else "bounds check clean", flush=True)
    return 1 if bad else 0


if __name__ == "__main__":
    sys.exit(main())
