"""Benchmark of the reweighting hot path on one MI355X.

One step = one rwgt_eval over the whole g g -> t t~ g g workload: 1e6 RAMBO
events (sqrt(s) uniform in [500, 2000] GeV, massive tops, gluon cuts), the
original card (alpha_s = 0.118) as normaliser and one new card
(alpha_s = 0.130): ingest of the momenta, |M|^2 under both cards for every
event, and w' = (w / |M|^2) * |M'|^2.  Inputs are resident in HBM before the
timed region.  The FP64 path gives ``value``; the mixed path (float
amplitudes) is timed the same way and reported under ``mixed``.  Both carry
the maximum relative error of w' against the exact ratio (0.130/0.118)^4 over
all events, which the oracle reproduces to 1e-13.

    python bench.py [--steps K] [--warmup W] [--events N] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "reweighted events/sec (gg→tt̄gg, FP64 vs mixed) at stated max rel. error"
RATIO = (0.130 / 0.118) ** 4
PEAK_FP64_VALU = 78.6e12        # MI355X FP64 vector, FLOP/s
PEAK_FP32_VALU_UNPACKED = 78.6e12  # 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz without packed FP32
# HBM bytes per launch of the matrix-element kernel, from the FETCH_SIZE and
# WRITE_SIZE counter passes (scaled by a copy kernel of known size); valid only
# for the kernel sources they were taken on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "me_kernel_gg_ttgg_1e6_traffic.json")
KERNEL_SOURCES = ["me_kernel.h", "kernels.h", "helas.h", "card.h", "check.h", "colour_mfma.h", "proc_gg_ttgg.hip",
                  "generated/gen_gg_ttgg.h"]


def kernel_sources_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2510_05100_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(mode, events):
    """Counter-measured HBM bytes per launch, or None when the counters were
    taken on other kernel sources, another mode or another event count."""
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    rec = d.get("modes", {}).get(mode)
    if not rec or d.get("sources_sha256") != kernel_sources_hash() or d.get("events") != events:
        return None
    return rec["bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--events", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2000)
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="oracle processes for the all-cores baseline (capped by the host's CPU count)")
    ap.add_argument("--modes", default="fp64,mixed")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-factored", action="store_true")
    ap.add_argument("--no-pcie", action="store_true", help="skip the pinned-host-memory (PCIe-inclusive) step")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the e+ e- -> mu+ mu- (1e4) and u u~ -> e+ e- g (1e6) legs")
    ap.add_argument("--surrogate-epochs", type=int, default=None,
                    help="training epochs of the surrogate networks (default: the Config default); fewer only "
                         "to keep a kernel trace short")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 512 MiB device copy (scale reference for HBM byte counters)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_mode(rw, torch, precision, p_dev, w_dev, rows, nevt, steps, warmup):
    import synth
    r = rw.Reweighter("g g > t t~ g g", synth.ORIG_QCD.slha(), precision)
    out = torch.empty((rows.shape[0], nevt), dtype=torch.float64, device="cuda")
    rw.rwgt_set_profiling(r.ctx, True)
    for _ in range(warmup):
        r.eval(p_dev, w_dev, rows, out)
    torch.cuda.synchronize()
    me_ms, ing_ms = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        r.eval(p_dev, w_dev, rows, out)
        a, b = rw.rwgt_kernel_times(r.ctx)
        ing_ms.append(a)
        me_ms.append(b)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    w = out.cpu().numpy()
    flops = rw.rwgt_flops(r.ctx)
    flops_exec = rw.rwgt_flops_executed(r.ctx)
    guard = rw.rwgt_mixed_guard_count(r.ctx)
    # |M|^2 under the original card (untimed), for the per-result errors
    me = torch.empty((1, nevt), dtype=torch.float64, device="cuda")
    r.me2(p_dev, synth.ORIG_QCD.row("gg_ttgg"), me)
    me = me.cpu().numpy()[0]
    r.close()
    rel = np.abs(w / RATIO - 1.0)
    return dict(ms_per_step=dt * 1e3, me_ms=float(np.mean(me_ms)), ingest_ms=float(np.mean(ing_ms)),
                max_rel_err=float(rel.max()), p999_rel_err=float(np.quantile(rel, 0.999)), flops_per_me2=flops,
                flops_exec_per_me2=flops_exec, w=w, me=me, reevaluated=guard)


def mixed_errors(rw, torch, p, p_dev, w_dev, rows, x, f, sample=200):
    """Errors of the mixed results per result kind: w' over every event
    against the exact ratio; |M|^2 over every event against the FP64 path (which
    agrees with the oracle to 1e-13) and on an evenly spaced sample against
    the oracle itself; and w' with the guard off, for comparison."""
    import synth
    from oracle import reweight
    me_rel = np.abs(x["me"] / f["me"] - 1.0)
    idx = np.linspace(0, p.shape[0] - 1, sample).astype(np.int64)
    ref = reweight.me2("gg_ttgg", p[idx], synth.ORIG_QCD)
    with rw.Reweighter("g g > t t~ g g", synth.ORIG_QCD.slha(), rw.RWGT_MIXED_FP16) as r:
        rw.rwgt_set_mixed_guard(r.ctx, 0.0)
        out = torch.empty((1, p.shape[0]), dtype=torch.float64, device="cuda")
        r.eval(p_dev, w_dev, rows, out)
        plain = np.abs(out.cpu().numpy() / RATIO - 1.0)
    return {"w_max_rel_err": x["max_rel_err"], "w_p999_rel_err": x["p999_rel_err"],
            "me2_max_rel_err_vs_fp64_path": float(me_rel.max()),
            "me2_p999_rel_err_vs_fp64_path": float(np.quantile(me_rel, 0.999)),
            "me2_max_rel_err_vs_oracle": float(np.max(np.abs(x["me"][idx] / ref - 1.0))),
            "oracle_sample": f"{sample} evenly spaced events",
            "w_max_rel_err_guard_off": float(plain.max())}


def workload_leg(rw, torch, proc, orig, new, n, steps, warmup, oracle_sample):
    """One of the other workloads at its own size (e+ e- -> mu+ mu-, 1e4
    events; u u~ -> e+ e- g, 1e6 events; g g -> t t~ t t~, 1e6 events; one new
    card), FP64 and mixed:
    reweighted events/s of the same timed rwgt_eval step as the headline,
    errors of w' and |M|^2 against the oracle on an evenly spaced sample, the
    mixed w' against the FP64 path on every event, and the FLOP rate of the
    matrix-element launch against the vector FP64 (FP32) peak."""
    import synth
    from oracle import reweight
    text = synth.PROCESSES[proc]
    p = synth.events(proc, n)
    p_dev = torch.as_tensor(p).cuda()
    w_dev = torch.ones(n, dtype=torch.float64, device="cuda")
    rows = new.row(proc)[None, :]
    idx = np.linspace(0, n - 1, min(n, oracle_sample)).astype(np.int64)
    ref_w, ref_me, _ = reweight.reweight(proc, p[idx], np.ones(idx.size), orig, [new])
    out, legs = {}, {}
    for mode, prec in (("fp64", rw.RWGT_FP64), ("mixed", rw.RWGT_MIXED_FP16)):
        r = rw.Reweighter(text, orig.slha(), prec)
        w = torch.empty((1, n), dtype=torch.float64, device="cuda")
        me = torch.empty((1, n), dtype=torch.float64, device="cuda")
        rw.rwgt_set_profiling(r.ctx, True)
        for _ in range(warmup):
            r.eval(p_dev, w_dev, rows, w)
        torch.cuda.synchronize()
        me_ms = []
        t0 = time.perf_counter()
        for _ in range(steps):
            r.eval(p_dev, w_dev, rows, w)
            me_ms.append(rw.rwgt_kernel_times(r.ctx)[1])
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        guard = rw.rwgt_mixed_guard_count(r.ctx)
        r.me2(p_dev, orig.row(proc), me)
        flops = rw.rwgt_flops(r.ctx) * n * 2
        flops_exec = rw.rwgt_flops_executed(r.ctx) * n * 2
        r.close()
        wh, meh = w.cpu().numpy()[0], me.cpu().numpy()[0]
        out[mode] = wh
        kernel_ms = float(np.mean(me_ms))
        legs[mode] = {"ms_per_step": dt * 1e3, "value": n / dt, "me_kernel_ms": kernel_ms,
                      "w_max_rel_err_vs_oracle": float(np.max(np.abs(wh[idx] / ref_w[0] - 1.0))),
                      "me2_max_rel_err_vs_oracle": float(np.max(np.abs(meh[idx] / ref_me - 1.0))),
                      "roofline": {"bound": "alu", "achieved": flops / (kernel_ms * 1e-3) / 1e12, "peak": 78.6,
                                   "unit": "TFLOP/s", "frac": flops / (kernel_ms * 1e-3) / PEAK_FP64_VALU,
                                   "executed_frac": flops_exec / (kernel_ms * 1e-3) / PEAK_FP64_VALU}}
        if mode == "mixed":
            rel = np.abs(wh / out["fp64"] - 1.0)
            legs[mode].update({"w_max_rel_err_vs_fp64_path": float(rel.max()),
                               "w_p999_rel_err_vs_fp64_path": float(np.quantile(rel, 0.999)),
                               "guard_reevaluated": guard})
    return {"workload": f"{text}, {n} events, 1 new card", "events": n, "oracle_sample": int(idx.size),
            "unit": "reweighted events/s", **legs}


def _limit_threads():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover
        pass


def _oracle_chunk(args):
    p, sl = args
    import synth
    from oracle import reweight
    w, _, _ = reweight.reweight("gg_ttgg", p[sl], np.ones(p[sl].shape[0]), synth.ORIG_QCD, [synth.NEW_QCD])
    return w[0]


def cpu_oracle(p, sample, workers):
    """The oracle as it stands on bounded samples of the same events, timed
    on one host core and on `workers` processes (one core each, the sample
    split into contiguous chunks).  Runs before the GPU is touched, so the
    worker processes are forks of a process without any GPU state."""
    import multiprocessing
    _limit_threads()
    idx = np.linspace(0, p.shape[0] - 1, sample).astype(np.int64)
    t0 = time.perf_counter()
    w1 = _oracle_chunk((p[idx], slice(None)))
    dt1 = time.perf_counter() - t0
    res = {"idx": idx, "w": w1, "single": sample / dt1, "single_s": dt1, "workers": 1}
    if workers > 1:
        n_mt = 4 * sample
        pm = p[np.linspace(0, p.shape[0] - 1, n_mt).astype(np.int64)]
        bounds = np.linspace(0, n_mt, workers + 1).astype(np.int64)     # one chunk per worker
        chunks = [(pm, slice(int(a), int(b))) for a, b in zip(bounds[:-1], bounds[1:])]
        try:
            with multiprocessing.get_context("fork").Pool(workers, initializer=_limit_threads) as pool:
                pool.map(_oracle_chunk, [(pm, slice(0, 1))] * workers)   # start the workers, import the oracle
                t0 = time.perf_counter()
                pool.map(_oracle_chunk, chunks)
                dtm = time.perf_counter() - t0
            res.update({"multi": n_mt / dtm, "multi_s": dtm, "multi_sample": n_mt, "workers": workers})
        except Exception as ex:  # pragma: no cover
            log(f"multi-process oracle timing skipped: {ex}")
    return res


def host_cpu():
    """(CPU model, logical CPUs of the host, CPUs this process may use)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return model, os.cpu_count() or 1, usable


def cpu_baseline(res, total, gpu_w):
    """The cpu_baseline object: the all-cores rate when it was measured (else
    the single-core one), with the single-core figure beside it, and the
    sampled parity of the GPU path against the oracle.  The all-cores run
    uses one single-thread process per core of this process's CPU share
    (capped by --cpu-workers, 16 by default: the host share of one GPU)."""
    idx, w = res["idx"], res["w"]
    model, logical, usable = host_cpu()
    host = {"cpu_model": model, "host_logical_cpus": logical, "cpus_usable_by_this_process": usable}
    parity = float(np.max(np.abs(gpu_w[0, idx] / w - 1.0)))
    single = (f"single core: {idx.size} events (evenly spaced) in {res['single_s']:.1f} s, "
              f"{res['single']:.1f} reweighted events/s")
    if res["workers"] > 1 and "multi" in res:
        return {"value": res["multi"], "unit": "reweighted events/s", "cores": res["workers"], "kind": "oracle",
                "sample": f"{res['multi_sample']} of the {total} g g -> t t~ g g events (evenly spaced), original + "
                          f"1 new card, FP64 numpy Berends-Giele oracle, {res['workers']} processes of one thread "
                          f"each, {res['multi_s']:.1f} s; {single}",
                "single_core_value": res["single"], "gpu_vs_oracle_max_rel_err": parity, **host}
    return {"value": res["single"], "unit": "reweighted events/s", "cores": 1, "kind": "oracle",
            "sample": f"{idx.size} of the {total} g g -> t t~ g g events (evenly spaced), original + 1 new card, "
                      f"FP64 numpy Berends-Giele oracle, single thread, {res['single_s']:.1f} s",
            "single_core_value": res["single"], "gpu_vs_oracle_max_rel_err": parity, **host}


def pcie_inclusive(rw, torch, p, rows, events, steps):
    """The FP64 step with the momenta, the weights and the output in pinned
    host memory, handed to rwgt_eval as they are: the library stages them
    through device memory on its stream (host-to-device copies, the same
    kernels, the device-to-host copy of w'), all timed together.  `value`
    is the device-resident rate; this one is reported beside it."""
    host_p = torch.as_tensor(p).pin_memory()
    host_w = torch.ones(events, dtype=torch.float64).pin_memory()
    out = torch.empty((rows.shape[0], events), dtype=torch.float64).pin_memory()
    ms = []
    with rw.Reweighter("g g > t t~ g g", __import__("synth").ORIG_QCD.slha(), rw.RWGT_FP64) as r:
        for i in range(steps + 1):
            s, e = (torch.cuda.Event(enable_timing=True) for _ in range(2))
            s.record()
            r.eval(host_p, host_w, rows, out, stream=torch.cuda.current_stream())
            e.record()
            torch.cuda.synchronize()
            if i:                                  # the first pass warms up
                ms.append(s.elapsed_time(e))
    step = float(np.mean(ms))
    h2d = host_p.numel() * 8 + host_w.numel() * 8
    return {"ms_per_step": step, "h2d_bytes": h2d, "d2h_bytes": out.numel() * 8,
            "value": events * rows.shape[0] / (step * 1e-3), "unit": "reweighted events/s"}


def batched_leg(rw, torch, precision, steps, warmup):
    """Config-3 style mix: 64 cards on the (M_Z, Gamma_Z, sin^2 theta_W) grid,
    each reweighting the first n events of a 2e5-event pool of e+e- -> mu+mu-
    and of u u~ -> e+e- g (n log-uniform in [1e3, 2e5], seeded): one tuned,
    graph-captured persistent launch against 128 separate rwgt_eval calls."""
    import synth
    grid = synth.batch_grid()
    counts = synth.batch_counts()
    procs = ("ee_mumu", "uu_eeg")
    texts = {"ee_mumu": "e+ e- > mu+ mu-", "uu_eeg": "u u~ > e+ e- g"}
    pools = {p: torch.as_tensor(synth.events(p, 200_000)).cuda() for p in procs}
    ones = torch.ones(200_000, dtype=torch.float64, device="cuda")
    ctxs = [rw.rwgt_create(texts[p], synth.ORIG_EW.slha(), precision) for p in procs]
    for ctx in ctxs:                      # the batched form runs unguarded: compare with the unguarded plain path
        rw.rwgt_set_mixed_guard(ctx, 0.0)
    items, plain_out = [], []
    for c, card in enumerate(grid):
        for j, p in enumerate(procs):
            n = int(counts[c, j])
            items.append((j, pools[p][:n], ones[:n], card.row(p), torch.empty(n, dtype=torch.float64, device="cuda")))
            plain_out.append(torch.empty((1, n), dtype=torch.float64, device="cuda"))
    total = int(counts.sum())
    b = rw.rwgt_batch_create(ctxs)
    segs, keep = rw.make_segments(items)
    t = time.perf_counter()
    sched = rw.rwgt_batch_tune(b, segs, reps=2)
    tune_s = time.perf_counter() - t
    for _ in range(warmup):
        rw.rwgt_batch_eval(b, segs)
    torch.cuda.synchronize()
    t = time.perf_counter()
    kernel_ms = []
    for _ in range(steps):
        rw.rwgt_batch_eval(b, segs)
        kernel_ms.append(rw.rwgt_batch_time(b))
    torch.cuda.synchronize()
    batched_ms = (time.perf_counter() - t) / steps * 1e3
    for ctx in ctxs:
        rw.rwgt_set_stream(ctx, None)

    def plain():
        for (j, mom, w, row, _), out in zip(items, plain_out):
            rw.rwgt_eval(ctxs[j], mom, w, row, out)
    for _ in range(warmup):
        plain()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        plain()
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t) / steps * 1e3
    diff = max(float(torch.max(torch.abs(it[4] - po[0]) / torch.abs(po[0])).item()) for it, po in zip(items, plain_out))
    rw.rwgt_batch_destroy(b)
    for ctx in ctxs:
        rw.rwgt_destroy(ctx)
    return {"events": total, "segments": len(items), "batched_ms": batched_ms,
            "batched_kernel_ms": float(np.mean(kernel_ms)), "plain_ms": plain_ms,
            "batched_value": total / (batched_ms * 1e-3), "plain_value": total / (plain_ms * 1e-3),
            "speedup": plain_ms / batched_ms, "schedule": sched, "tune_seconds": tune_s,
            "max_rel_diff_vs_plain": diff, "unit": "reweighted events/s"}


def factored_leg(rw, torch, steps, warmup, n=1_000_000):
    """u u~ -> e+ e- g, n events x the 64-card grid: the full path (1 + 64
    matrix-element evaluations per event) against the coupling-factored path
    (4 probe evaluations per event, then a few operations per card)."""
    import synth
    p = synth.events("uu_eeg", n)
    rows = np.stack([c.row("uu_eeg") for c in synth.batch_grid()])
    p_dev = torch.as_tensor(p).cuda()
    w_dev = torch.ones(n, dtype=torch.float64, device="cuda")
    full = torch.empty((rows.shape[0], n), dtype=torch.float64, device="cuda")
    fac = torch.empty_like(full)
    r = rw.Reweighter("u u~ > e+ e- g", synth.ORIG_EW.slha())

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps * 1e3
    full_ms = timed(lambda: r.eval(p_dev, w_dev, rows, full))
    fac_ms = timed(lambda: r.eval_factored(p_dev, w_dev, rows, fac))
    diff = float(torch.max(torch.abs(fac - full) / torch.abs(full)).item())
    r.close()
    pairs = n * rows.shape[0]
    return {"events": n, "cards": int(rows.shape[0]), "full_ms": full_ms, "factored_ms": fac_ms,
            "full_value": pairs / (full_ms * 1e-3), "factored_value": pairs / (fac_ms * 1e-3),
            "speedup": full_ms / fac_ms, "max_rel_diff": diff, "unit": "reweighted (event, card) pairs/s"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the events are independent "
              "and a multi-GPU run would shard them without any exchange in the hot path.", file=sys.stderr)
        sys.exit(2)
    import synth
    t = time.perf_counter()
    p = synth.events("gg_ttgg", a.events)
    log(f"generated {a.events} events in {time.perf_counter() - t:.1f}s")
    oracle_res = None
    if not a.no_cpu_baseline:                 # host cores first, before any GPU state exists
        oracle_res = cpu_oracle(p, a.cpu_sample, max(1, min(a.cpu_workers, host_cpu()[2])))
        log(f"oracle: {oracle_res['single']:.1f} events/s on one core" +
            (f", {oracle_res['multi']:.1f} on {oracle_res['workers']}" if "multi" in oracle_res else ""))
    import torch
    import paper_2510_05100_amd as rw
    rw.load()
    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    p_dev = torch.as_tensor(p).cuda()
    w_dev = torch.ones(a.events, dtype=torch.float64, device="cuda")
    rows = synth.NEW_QCD.row("gg_ttgg")[None, :]
    res = {}
    for mode in a.modes.split(","):
        prec = rw.RWGT_FP64 if mode == "fp64" else rw.RWGT_MIXED_FP16
        res[mode] = time_mode(rw, torch, prec, p_dev, w_dev, rows, a.events, a.steps, a.warmup)
        log(f"{mode}: {res[mode]['ms_per_step']:.2f} ms/step, ME kernel {res[mode]['me_ms']:.2f} ms, "
            f"max rel err {res[mode]['max_rel_err']:.3g}")
    nsets = rows.shape[0]

    def roofline(r, peak, mode):
        # algorithmic: the plain per-helicity sum over all 64 kept helicities;
        # executed: the 32 the kernel evaluates (|M_h|^2 = |M_~h|^2 in QCD)
        flops = r["flops_per_me2"] * a.events * (1 + nsets)
        flops_exec = r["flops_exec_per_me2"] * a.events * (1 + nsets)
        ach = flops / (r["me_ms"] * 1e-3)
        ach_exec = flops_exec / (r["me_ms"] * 1e-3)
        return {"bound": "alu", "achieved": ach / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": ach / peak, "traffic": measured_traffic(mode, a.events),
                "kernel": "me_kernel<Proc_gg_ttgg>", "flops_per_launch": flops,
                "executed_flops_per_launch": flops_exec, "executed_achieved": ach_exec / 1e12,
                "executed_frac": ach_exec / peak,
                "flops_definition": "achieved/frac: the plain per-helicity sum over all 64 helicities (rwgt_flops); "
                                    "executed_*: the 32 the kernel evaluates, one of each pair with every helicity "
                                    "reversed, whose |M_h|^2 are equal in QCD (rwgt_flops_executed)"}

    main_mode = "fp64" if "fp64" in res else next(iter(res))
    m = res[main_mode]
    value = a.events * nsets / (m["ms_per_step"] * 1e-3)
    line = {
        "metric": METRIC, "value": value, "unit": "reweighted events/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if main_mode == "fp64" else "f32", "data": "synthetic",
        "config": {"workload": f"g g -> t t~ g g, {a.events} RAMBO events (sqrt(s) in [500, 2000] GeV, "
                               "pT(g) > 30 GeV, dR(g,g) > 0.4), alpha_s 0.118 -> 0.130, 1 new card",
                   "events": a.events, "new_cards": nsets, "precision": main_mode},
        "max_rel_err": m["max_rel_err"],
        "roofline": roofline(m, PEAK_FP64_VALU, main_mode),
    }
    if "mixed" in res and main_mode != "mixed":
        x = res["mixed"]
        line["mixed"] = {"value": a.events * nsets / (x["ms_per_step"] * 1e-3), "ms_per_step": x["ms_per_step"],
                         "max_rel_err": x["max_rel_err"], "dtype": "f32 amplitudes, f64 momenta/denominators/ratio",
                         "roofline": roofline(x, PEAK_FP32_VALU_UNPACKED, "mixed"),
                         "guard": {"kappa_max": 300.0, "reevaluated_fp64": x["reevaluated"],
                                   "fraction": x["reevaluated"] / a.events},
                         "errors": mixed_errors(rw, torch, p, p_dev, w_dev, rows, x, m)}
    if not a.no_workloads:
        line["workloads"] = {}
        for key, proc, orig, new, n, sample in (("ee_mumu_1e4", "ee_mumu", synth.ORIG_EW, synth.NEW_EE, 10_000, 10_000),
                                                ("uu_eeg_1e6", "uu_eeg", synth.ORIG_EW, synth.NEW_UU, 1_000_000, 1000),
                                                ("gg_tttt_1e6", "gg_tttt", synth.ORIG_QCD, synth.NEW_QCD, 1_000_000, 6)):
            line["workloads"][key] = workload_leg(rw, torch, proc, orig, new, n, steps=a.steps, warmup=a.warmup,
                                                  oracle_sample=sample)
            log(f"{key}: fp64 {line['workloads'][key]['fp64']['value']:.3g}, mixed "
                f"{line['workloads'][key]['mixed']['value']:.3g} reweighted events/s")
    if main_mode == "fp64" and not a.no_pcie:
        line["pcie_inclusive"] = pcie_inclusive(rw, torch, p, rows, a.events, steps=3)
        log(f"pcie-inclusive: {line['pcie_inclusive']['ms_per_step']:.2f} ms/step")
    if not a.no_batched:
        line["batched"] = {}
        for mode, prec in (("fp64", rw.RWGT_FP64), ("mixed", rw.RWGT_MIXED_FP16)):
            line["batched"][mode] = batched_leg(rw, torch, prec, steps=5, warmup=2)
            log(f"batched {mode}: {line['batched'][mode]['batched_ms']:.2f} ms vs plain "
                f"{line['batched'][mode]['plain_ms']:.2f} ms")
    if not a.no_factored:
        line["factored"] = factored_leg(rw, torch, steps=5, warmup=2)
        log(f"factored: {line['factored']['factored_ms']:.2f} ms vs full {line['factored']['full_ms']:.2f} ms")
    if not a.no_surrogate:
        # the workload's network (raw momenta + card, 4 x 256) and the
        # physics-feature network (18 inputs, 3 x 128), same data and gate
        from paper_2510_05100_amd import surrogate
        line["surrogate"] = {}
        for name, cfg in (("raw_23_4x256", surrogate.Config(width=256, depth=4, features=rw.RWGT_FEAT_RAW)),
                          ("physics_18_3x128", surrogate.Config())):
            if a.surrogate_epochs:
                cfg.epochs = a.surrogate_epochs
            summary, sur = surrogate.run(torch, cfg, log=log)
            sur.close()
            line["surrogate"][name] = summary
    if a.copy_probe:
        src = torch.empty(64 << 20, dtype=torch.float64, device="cuda")
        dst = src.clone()
        torch.cuda.synchronize()
        line["copy_probe_bytes"] = 2 * src.numel() * 8
        del src, dst
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(oracle_res, a.events, m["w"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
