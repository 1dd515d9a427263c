"""Reweighting of a Les Houches event file, the way the paper's MadtRex
executables run it: read the file, sort its events into the supported
processes, reweight each process's events on the GPU for every parameter set
of a reweighting card, and write the file back with one new weight per set
(0 for events of processes that are not evaluated).  The file work happens in
the library's host code (rwgt_lhe_*, rwgt_reweight_card), the arithmetic in
its kernels (rwgt_eval or rwgt_eval_factored); this module sequences the
calls and moves arrays between host and device.
"""
from __future__ import annotations

import time

import numpy as np

from . import _abi

PROCESSES = ("e+ e- > mu+ mu-", "u u~ > e+ e- g", "g g > t t~ g g", "g g > t t~ t t~")
# The reweighting card's "change fptype": d is FP64 and f single-precision
# amplitudes (the library's mixed mode).  The paper's default m keeps the
# amplitudes in FP64 and only the colour algebra in FP32; it runs here as FP64
# (no FP32 amplitudes: at least as accurate, and the FP64 colour sum costs
# about a tenth of the evaluation on these vector units).
FPTYPE = {"d": _abi.RWGT_FP64, "f": _abi.RWGT_MIXED_FP16, "m": _abi.RWGT_FP64}


def reweight_lhe(in_path, out_path, param_card, rwgt_card, precision=None, factored=False, running_alphas=False,
                 log=None):
    """Reweight every supported process in in_path; write out_path.

    param_card: SLHA text of the original card; rwgt_card: reweighting-card
    text ("launch rwgt_name=..." / "set BLOCK ID VALUE").  precision: an
    RWGT_* constant, else the card's "change fptype" (d or m: FP64; f:
    mixed), else FP64.  factored: use the coupling-factored path.  running_alphas:
    the strong coupling per event (the event's AQCDUP for the original card,
    each card's alpha_s run to the event's SCALUP; rwgt_eval_alphas).
    Returns a summary
    (events per process, weight names, seconds per stage)."""
    import torch
    t0 = time.perf_counter()
    lhe = _abi.rwgt_lhe_read(in_path)
    summary = {"events": 0, "processes": {}, "weights": [], "read_s": 0.0, "eval_s": 0.0, "write_s": 0.0}
    try:
        summary["events"] = _abi.rwgt_lhe_num_events(lhe)
        summary["read_s"] = time.perf_counter() - t0
        names_all = []
        for proc in PROCESSES:
            idx = _abi.rwgt_lhe_select(lhe, proc)
            sets, names, fp = _abi.rwgt_reweight_card(proc, param_card, rwgt_card)
            for nm in names:
                if nm not in names_all:
                    names_all.append(nm)
            if idx.size == 0 or len(names) == 0:
                continue
            prec = precision if precision is not None else FPTYPE.get(fp or "d", _abi.RWGT_FP64)
            mom, w = _abi.rwgt_lhe_momenta(lhe, proc, idx)
            t1 = time.perf_counter()
            ctx = _abi.rwgt_create(proc, param_card, prec)
            try:
                _abi.rwgt_set_stream(ctx, None)
                p_dev = torch.as_tensor(mom).cuda()
                w_dev = torch.as_tensor(w).cuda()
                out = torch.empty((sets.shape[0], idx.size), dtype=torch.float64, device="cuda")
                if running_alphas:
                    info = _abi.rwgt_lhe_info(lhe, idx)
                    aqcd = torch.as_tensor(np.ascontiguousarray(info[:, 3])).cuda()
                    scale = torch.as_tensor(np.ascontiguousarray(info[:, 1])).cuda()
                    _abi.rwgt_eval_alphas(ctx, p_dev, w_dev, aqcd, scale, sets, out)
                else:
                    (_abi.rwgt_eval_factored if factored else _abi.rwgt_eval)(ctx, p_dev, w_dev, sets, out)
                wn = out.cpu().numpy()
            finally:
                _abi.rwgt_destroy(ctx)
            summary["eval_s"] += time.perf_counter() - t1
            for k, nm in enumerate(names):
                _abi.rwgt_lhe_add_weights(lhe, nm, nm, idx, wn[k])
            summary["processes"][proc] = int(idx.size)
            if log:
                log(f"{proc}: {idx.size} events x {len(names)} sets")
        # every set gets a weight, also when no event of the file was evaluated
        empty = np.zeros(0, dtype=np.int64)
        for nm in names_all:
            _abi.rwgt_lhe_add_weights(lhe, nm, nm, empty, np.zeros(0))
        summary["weights"] = names_all
        t2 = time.perf_counter()
        _abi.rwgt_lhe_write(lhe, out_path)
        summary["write_s"] = time.perf_counter() - t2
    finally:
        _abi.rwgt_lhe_destroy(lhe)
    return summary
