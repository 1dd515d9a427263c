"""Learned surrogate for the reweighting ratio of u u~ -> e+ e- g.

A network maps an (event, card) pair to mu = log(w'/w) and to s, the log of
the error of mu.  Inputs: the physics feature map (log s_hat, the ten pair
invariants log(s_ij / s_hat), the card's M_Z, Gamma_Z, sin^2 theta_W, and
asinh of the real and imaginary parts of the Z-to-photon propagator ratio of
the lepton pair under the card and under the original card: 18 inputs), or
the raw map (momenta and card, 23 inputs).  It is trained on ratios from the
exact matrix-element path and used with an exact fallback: where the
calibrated error bound k exp(s) exceeds a threshold the event is reweighted
exactly (rwgt_sur_eval).  Every step of training and inference runs in the
library (features, normalisation statistics, the shuffled epoch loop with its
learning-rate schedule, forward, backward, Adam, the calibration quantile,
checkpoints, fused inference and gate); this module only sequences the calls
and keeps the timings.

Workload: 64 cards on the (M_Z, Gamma_Z, sin^2 theta_W) grid; training on
62,500 events x 64 cards = 4e6 (event, card) pairs (seed 3000); calibration on
a separate 62,500 x 64 set (seed 3002); held-out evaluation on 1e6 fresh
events (seed 3001), each with a uniformly drawn grid card.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import _abi

PROCESS = "u u~ > e+ e- g"
NPART = 5
RESONANT_PAIR = (2, 3)          # e+ e-
SEED_CALIBRATION = 3002


@dataclasses.dataclass
class Config:
    width: int = 128
    depth: int = 3
    precision: int = _abi.RWGT_MLP_BF16
    features: int = _abi.RWGT_FEAT_PHYS
    batch: int = 4096
    epochs: int = 250
    lr: float = 2e-3
    lr_final: float = 2e-5
    lam: float = 0.001
    seed: int = 1
    coverage: float = 0.999     # quantile of |r| / exp(s) taken as k


def card_table(cards, process="uu_eeg"):
    """(param_sets rows [n][npar] float64, network card inputs [n][3] float32)."""
    rows = np.stack([c.row(process) for c in cards])
    net = np.array([[c.MZ, c.WZ, c.sw2] for c in cards], dtype=np.float32)
    return rows, net


def exact_ratios(ctx, torch, mom_dev, rows):
    """w'[card][event] from the exact path for unit input weights."""
    n = mom_dev.shape[0]
    ones = torch.ones(n, dtype=torch.float64, device="cuda")
    out = torch.empty((rows.shape[0], n), dtype=torch.float64, device="cuda")
    _abi.rwgt_set_stream(ctx, None)
    _abi.rwgt_eval(ctx, mom_dev, ones, rows, out)
    return out


class Surrogate:
    def __init__(self, cfg: Config | None = None, orig=None):
        import synth
        self.cfg = cfg or Config()
        self.orig = orig or (synth.ORIG_EW.MZ, synth.ORIG_EW.WZ)
        self.n_in = _abi.n_features(self.cfg.features, NPART)
        self.mlp = _abi.rwgt_mlp_create(self.n_in, self.cfg.width, self.cfg.depth, 2, self.cfg.precision,
                                        self.cfg.seed)
        _abi.rwgt_mlp_set_features(self.mlp, self.cfg.features, NPART, RESONANT_PAIR, self.orig)
        _abi.rwgt_mlp_set_training(self.mlp, self.cfg.lam)
        self.k = None
        self.history = []

    def close(self):
        if self.mlp:
            _abi.rwgt_mlp_destroy(self.mlp)
            self.mlp = None

    # ------------------------------------------------------------- training
    def fit(self, torch, mom_dev, net_cards_dev, y_dev, n_events, n_cards, log=print, epochs_per_call=25):
        """y_dev: log ratios [n_cards][n_events] (float32, device).  The
        library fits the normalisations and runs the epochs (shuffle, features,
        forward, backward, Adam, learning-rate schedule); this loop only
        asks for them in pieces to log the loss."""
        cfg = self.cfg
        _abi.rwgt_mlp_set_stream(self.mlp, None)
        assert mom_dev.shape[0] == n_events and y_dev.shape == (n_cards, n_events)
        if _abi.rwgt_mlp_get_progress(self.mlp)[0] == 0:
            _abi.rwgt_mlp_fit_grid(self.mlp, mom_dev, net_cards_dev, y_dev)
        t0 = time.perf_counter()
        done = _abi.rwgt_mlp_get_progress(self.mlp)[0]
        while done < cfg.epochs:
            end = min(cfg.epochs, done + epochs_per_call)
            losses = _abi.rwgt_mlp_train(self.mlp, mom_dev, net_cards_dev, y_dev, cfg.batch, cfg.epochs, cfg.lr,
                                         cfg.lr_final, cfg.seed, end)
            for k, v in enumerate(losses):
                self.history.append(float(v))
                log(f"epoch {done + k}: mean loss {v:.4g} ({time.perf_counter() - t0:.1f}s)")
            done = end
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def predict(self, torch, mom_dev, card_index_dev, net_cards_dev, event_index_dev=None):
        """(mu, s) for each row from the fused kernel (device float32 tensors)."""
        n = card_index_dev.shape[0]
        heads = torch.empty((n, 2), dtype=torch.float32, device="cuda")
        _abi.rwgt_mlp_set_stream(self.mlp, None)
        _abi.rwgt_mlp_predict(self.mlp, mom_dev, event_index_dev, card_index_dev, net_cards_dev, n, heads)
        return heads[:, 0], heads[:, 1]

    def calibrate(self, torch, mom_dev, net_cards_dev, y_dev, n_events, n_cards):
        """k = coverage quantile of |y - mu| / exp(s) over the calibration pairs (in the library)."""
        assert mom_dev.shape[0] == n_events and y_dev.shape == (n_cards, n_events)
        k, med, p90, p999 = _abi.rwgt_mlp_calibrate(self.mlp, mom_dev, net_cards_dev, y_dev, self.cfg.coverage)
        self.k = k
        return {"k": k, "median_abs_err": med, "p90_abs_err": p90, "p999_abs_err": p999}

    # ---------------------------------------------------------- checkpoints
    def save(self, path):
        """Everything a resumed run needs (library checkpoint: parameters, Adam
        moments and step count, schedule and epoch, normalisations, k)."""
        _abi.rwgt_mlp_save(self.mlp, path)

    @classmethod
    def load(cls, path, cfg: Config | None = None):
        """A surrogate from a checkpoint; cfg (optional) carries the training
        schedule to resume with (it must match the saved one)."""
        shape, _, _ = _abi.rwgt_mlp_checkpoint_info(path)
        n_in, width, depth, _, precision = shape
        s = cls.__new__(cls)
        s.cfg = cfg or Config(width=width, depth=depth, precision=precision)
        s.mlp = _abi.rwgt_mlp_load(path)
        s.n_in = n_in
        s.orig = None
        s.k = None
        s.history = []
        return s


def run(torch, cfg: Config | None = None, n_train=62_500, n_heldout=1_000_000, threshold=1e-3, log=print):
    """Train, calibrate and evaluate; returns (summary, surrogate)."""
    import synth
    cfg = cfg or Config()
    grid = synth.batch_grid()
    rows, net_cards = card_table(grid)
    ctx = _abi.rwgt_create(PROCESS, synth.ORIG_EW.slha(), _abi.RWGT_FP64)
    sur = Surrogate(cfg)
    try:
        ncards = len(grid)
        p_train = synth.events("uu_eeg", n_train, seed=synth.workloads.SEED_SUR_TRAIN)
        p_cal = synth.events("uu_eeg", n_train, seed=SEED_CALIBRATION)
        mom_t = torch.as_tensor(p_train).cuda()
        mom_c = torch.as_tensor(p_cal).cuda()
        net_dev = torch.as_tensor(net_cards).cuda()
        t0 = time.perf_counter()
        y_t = torch.empty((ncards, n_train), dtype=torch.float32, device="cuda")
        y_c = torch.empty((ncards, n_train), dtype=torch.float32, device="cuda")
        _abi.rwgt_mlp_set_stream(sur.mlp, None)
        _abi.rwgt_mlp_targets(sur.mlp, exact_ratios(ctx, torch, mom_t, rows), None, y_t)
        _abi.rwgt_mlp_targets(sur.mlp, exact_ratios(ctx, torch, mom_c, rows), None, y_c)
        torch.cuda.synchronize()
        data_s = time.perf_counter() - t0
        train_s = sur.fit(torch, mom_t, net_dev, y_t, n_train, ncards, log=log)
        cal = sur.calibrate(torch, mom_c, net_dev, y_c, n_train, ncards)
        log(f"calibration: {cal}")
        summary = {"features": "physics" if cfg.features == _abi.RWGT_FEAT_PHYS else "raw",
                   "network": f"{sur.n_in}-{'-'.join([str(cfg.width)] * cfg.depth)}-2",
                   "train_pairs": n_train * ncards, "epochs": cfg.epochs, "data_seconds": data_s,
                   "train_seconds": train_s, "final_loss": sur.history[-1], "calibration": cal}
        summary.update(evaluate(torch, ctx, sur, rows, net_dev, n_heldout, threshold, log=log))
        return summary, sur
    finally:
        _abi.rwgt_destroy(ctx)


def evaluate(torch, ctx, sur, rows, net_dev, n_heldout, threshold, log=print, reps=5, extra_thresholds=(1e-2,)):
    """Surrogate path (with exact fallback) against the exact card-per-event
    path on held-out events with uniformly drawn cards."""
    import synth
    p = synth.events("uu_eeg", n_heldout, seed=synth.workloads.SEED_SUR_HELDOUT)
    cidx = synth.surrogate_cards(n_heldout).astype(np.int32)
    mom = torch.as_tensor(p).cuda()
    cd = torch.as_tensor(cidx).cuda()
    w = torch.ones(n_heldout, dtype=torch.float64, device="cuda")
    exact = torch.empty(n_heldout, dtype=torch.float64, device="cuda")
    sur_w = torch.empty(n_heldout, dtype=torch.float64, device="cuda")
    _abi.rwgt_set_stream(ctx, None)

    def timed(fn):
        r = fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps * 1e3, r

    exact_ms, _ = timed(lambda: _abi.rwgt_eval_cards(ctx, mom, w, rows, cd, exact))
    e = exact.cpu().numpy()
    # network only (fused features + layers + heads, no gate) for reference
    net_ms, _ = timed(lambda: sur.predict(torch, mom, cd, net_dev))
    points = []
    for thr in (threshold,) + tuple(extra_thresholds):
        sur_ms, nfb = timed(lambda: _abi.rwgt_sur_eval(ctx, sur.mlp, mom, w, rows, cd, thr, sur_w))
        s = sur_w.cpu().numpy()
        rel = np.abs(s / e - 1.0)
        points.append({"threshold": thr, "fallback": int(nfb), "fallback_fraction": nfb / n_heldout,
                       "max_rel_err": float(rel.max()), "p999_rel_err": float(np.quantile(rel, 0.999)),
                       "events_beyond_threshold": int(np.sum(rel > thr)), "surrogate_path_ms": sur_ms,
                       "gain": exact_ms / sur_ms, "surrogate_value": n_heldout / (sur_ms * 1e-3)})
    res = {"heldout_events": n_heldout, "exact_path_ms": exact_ms, "exact_value": n_heldout / (exact_ms * 1e-3),
           "network_only_ms": net_ms}
    res.update(points[0])
    res["other_thresholds"] = points[1:]
    log(f"held-out: {res}")
    return res
