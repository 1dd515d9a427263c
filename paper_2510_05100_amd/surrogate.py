"""Learned surrogate for the reweighting ratio of u u~ -> e+ e- g.

A network maps (the five four-momenta, M_Z, Gamma_Z, sin^2 theta_W) to
mu = log(w'/w) and to s, the log of the error of mu.  It is trained on ratios
produced by the exact matrix-element path and used with an exact fallback:
where the calibrated error bound k exp(s) exceeds a threshold the event is
reweighted exactly (rwgt_sur_eval).  Every numerical step runs in the
library's kernels; this module only sequences the calls (data set assembly,
shuffling, learning-rate schedule, calibration quantile, checkpoints).

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
N_IN = 23            # 5 x 4 momenta + 3 card parameters
SEED_CALIBRATION = 3002


@dataclasses.dataclass
class Config:
    width: int = 256
    depth: int = 4
    precision: int = _abi.RWGT_MLP_BF16
    batch: int = 4096
    epochs: int = 12
    lr: float = 2e-3
    lr_final: float = 2e-5
    lam: float = 0.1
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


def raw_feature_stats(p, net_cards):
    """Mean and standard deviation of the 23 raw inputs over the (event, card)
    pairs of the training set (host, float64)."""
    mom = p.reshape(p.shape[0], -1)
    mean = np.concatenate([mom.mean(axis=0), net_cards.mean(axis=0)])
    std = np.concatenate([mom.std(axis=0), net_cards.std(axis=0)])
    std[std == 0] = 1.0
    return mean.astype(np.float32), std.astype(np.float32)


class Surrogate:
    def __init__(self, cfg: Config | None = None):
        self.cfg = cfg or Config()
        self.mlp = _abi.rwgt_mlp_create(N_IN, self.cfg.width, self.cfg.depth, 2, self.cfg.precision, self.cfg.seed)
        _abi.rwgt_mlp_set_training(self.mlp, self.cfg.lam)
        self.k = None
        self.history = []

    def close(self):
        if self.mlp:
            _abi.rwgt_mlp_destroy(self.mlp)
            self.mlp = None

    # ------------------------------------------------------------- training
    def fit(self, torch, mom_dev, net_cards_dev, y_dev, n_events, n_cards, mean, std, log=print):
        """y_dev: log ratios [n_cards][n_events] (float32, device)."""
        cfg = self.cfg
        _abi.rwgt_mlp_set_stream(self.mlp, None)
        _abi.rwgt_mlp_set_normalisation(self.mlp, mean, std)
        total = n_events * n_cards
        steps_per_epoch = total // cfg.batch
        xbuf = torch.empty(_abi.rwgt_mlp_input_bytes(self.mlp, cfg.batch), dtype=torch.uint8, device="cuda")
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        yflat = y_dev.reshape(-1)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(cfg.seed)
        nsteps = steps_per_epoch * cfg.epochs
        t0 = time.perf_counter()
        step = 0
        for epoch in range(cfg.epochs):
            perm = torch.randperm(total, device="cuda", generator=gen)
            ev = (perm % n_events).to(torch.int32)
            cd = (perm // n_events).to(torch.int32)
            yp = yflat[perm].contiguous()
            acc = 0.0
            for b in range(steps_per_epoch):
                sl = slice(b * cfg.batch, (b + 1) * cfg.batch)
                lr = cfg.lr * (cfg.lr_final / cfg.lr) ** (step / max(1, nsteps - 1))
                _abi.rwgt_mlp_features(self.mlp, mom_dev, ev[sl], cd[sl], net_cards_dev, cfg.batch, xbuf)
                _abi.rwgt_mlp_train_step(self.mlp, xbuf, yp[sl], cfg.batch, lr, loss)
                if b % 64 == 0:
                    acc += float(loss.item()) / cfg.batch
                step += 1
            self.history.append(acc / ((steps_per_epoch + 63) // 64))
            log(f"epoch {epoch}: mean loss {self.history[-1]:.4g} ({time.perf_counter() - t0:.1f}s)")
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def predict(self, torch, mom_dev, card_index_dev, net_cards_dev, event_index_dev=None):
        """(mu, s) for each row, in chunks (device float32 tensors)."""
        n = card_index_dev.shape[0]
        chunk = 1 << 18
        mu = torch.empty(n, dtype=torch.float32, device="cuda")
        s = torch.empty(n, dtype=torch.float32, device="cuda")
        xbuf = torch.empty(_abi.rwgt_mlp_input_bytes(self.mlp, chunk), dtype=torch.uint8, device="cuda")
        heads = torch.empty((chunk, 32), dtype=torch.float32, device="cuda")
        _abi.rwgt_mlp_set_stream(self.mlp, None)
        for a in range(0, n, chunk):
            b = min(n, a + chunk)
            evi = None if event_index_dev is None else event_index_dev[a:b]
            mom = mom_dev if event_index_dev is not None else mom_dev[a:b]
            _abi.rwgt_mlp_features(self.mlp, mom, evi, card_index_dev[a:b], net_cards_dev, b - a, xbuf)
            _abi.rwgt_mlp_forward(self.mlp, xbuf, b - a, heads)
            mu[a:b] = heads[:b - a, 0]
            s[a:b] = heads[:b - a, 1]
        return mu, s

    def calibrate(self, torch, mom_dev, net_cards_dev, y_dev, n_events, n_cards):
        """k = quantile of |y - mu| / exp(s) over the calibration pairs."""
        total = n_events * n_cards
        idx = torch.arange(total, device="cuda")
        ev = (idx % n_events).to(torch.int32)
        cd = (idx // n_events).to(torch.int32)
        mu, s = self.predict(torch, mom_dev, cd, net_cards_dev, ev)
        z = (torch.abs(y_dev.reshape(-1) - mu) / torch.exp(s)).cpu().numpy()
        self.k = float(np.quantile(z, self.cfg.coverage))
        _abi.rwgt_mlp_set_calibration(self.mlp, self.k)
        resid = (y_dev.reshape(-1) - mu).abs().cpu().numpy()
        return {"k": self.k, "median_abs_err": float(np.median(resid)), "p999_abs_err": float(np.quantile(resid, 0.999))}

    # ---------------------------------------------------------- checkpoints
    def save(self, path, mean, std):
        np.savez(path, params=_abi.rwgt_mlp_get_params(self.mlp), mean=mean, std=std,
                 k=np.float64(self.k or 0.0), width=self.cfg.width, depth=self.cfg.depth,
                 precision=self.cfg.precision, history=np.array(self.history))

    @classmethod
    def load(cls, path):
        d = np.load(path)
        s = cls(Config(width=int(d["width"]), depth=int(d["depth"]), precision=int(d["precision"])))
        _abi.rwgt_mlp_set_params(s.mlp, d["params"])
        _abi.rwgt_mlp_set_normalisation(s.mlp, d["mean"], d["std"])
        if float(d["k"]) > 0:
            s.k = float(d["k"])
            _abi.rwgt_mlp_set_calibration(s.mlp, s.k)
        return s


def run(torch, cfg: Config | None = None, n_train=62_500, n_heldout=1_000_000, threshold=1e-3, log=print):
    """Train, calibrate and evaluate; returns a summary dictionary."""
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
        mean, std = raw_feature_stats(p_train, net_cards)
        train_s = sur.fit(torch, mom_t, net_dev, y_t, n_train, ncards, mean, std, log=log)
        cal = sur.calibrate(torch, mom_c, net_dev, y_c, n_train, ncards)
        log(f"calibration: {cal}")
        summary = {"train_pairs": n_train * ncards, "epochs": cfg.epochs, "data_seconds": data_s,
                   "train_seconds": train_s, "final_loss": sur.history[-1], "calibration": cal}
        summary.update(evaluate(torch, ctx, sur, rows, net_dev, n_heldout, threshold, log=log))
        return summary, sur, (mean, std)
    finally:
        _abi.rwgt_destroy(ctx)


def evaluate(torch, ctx, sur, rows, net_dev, n_heldout, threshold, log=print, reps=5):
    """Surrogate path (with exact fallback) against the exact path on held-out
    events with uniformly drawn cards."""
    import synth
    p = synth.events("uu_eeg", n_heldout, seed=synth.workloads.SEED_SUR_HELDOUT)
    cidx = synth.surrogate_cards(n_heldout).astype(np.int32)
    mom = torch.as_tensor(p).cuda()
    cd = torch.as_tensor(cidx).cuda()
    w = torch.ones(n_heldout, dtype=torch.float64, device="cuda")
    exact = torch.empty(n_heldout, dtype=torch.float64, device="cuda")
    sur_w = torch.empty(n_heldout, dtype=torch.float64, device="cuda")
    _abi.rwgt_set_stream(ctx, None)

    def timed(thr, out):
        nfb = _abi.rwgt_sur_eval(ctx, sur.mlp, mom, w, rows, cd, thr, out)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            nfb = _abi.rwgt_sur_eval(ctx, sur.mlp, mom, w, rows, cd, thr, out)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps * 1e3, nfb
    exact_ms, _ = timed(0.0, exact)          # threshold 0: every event exact
    sur_ms, nfb = timed(threshold, sur_w)
    e = exact.cpu().numpy()
    s = sur_w.cpu().numpy()
    rel = np.abs(s / e - 1.0)
    used = rel > 0
    # network-only throughput (features + forward) for reference
    mu, _ = sur.predict(torch, mom, cd, net_dev)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        sur.predict(torch, mom, cd, net_dev)
    torch.cuda.synchronize()
    net_ms = (time.perf_counter() - t) / reps * 1e3
    res = {"heldout_events": n_heldout, "threshold": threshold, "fallback": int(nfb),
           "fallback_fraction": nfb / n_heldout, "max_rel_err": float(rel.max()),
           "p999_rel_err": float(np.quantile(rel, 0.999)), "events_beyond_threshold": int(np.sum(rel > threshold)),
           "surrogate_path_ms": sur_ms, "exact_path_ms": exact_ms, "network_only_ms": net_ms,
           "gain": exact_ms / sur_ms, "surrogate_value": n_heldout / (sur_ms * 1e-3),
           "exact_value": n_heldout / (exact_ms * 1e-3), "n_network_evaluated": int(used.sum())}
    log(f"held-out: {res}")
    return res
