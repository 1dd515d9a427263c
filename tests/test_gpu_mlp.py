"""Surrogate network kernels against the FP64 reference network (oracle/mlp.py)
and the surrogate reweighting path against the exact one.

Tolerances: the FP32 form (VALU GEMM, FP32 activations) differs from the
FP64 reference by FP32 rounding accumulated over sums of at most 256 terms
per layer: 1e-5 relative on each layer's gradient norm and on the heads.  The
BF16 form rounds weights, activations and backpropagated gradients to 8
significant bits: 2e-2 relative.
"""
import numpy as np
import pytest

import synth
from oracle import mlp as omlp

from gpu_util import PROCESS_TEXT, dev, rel_err, torch_cuda

pytestmark = pytest.mark.gpu

N_IN, WIDTH, DEPTH = 23, 256, 4
SHAPES = [(WIDTH, N_IN)] + [(WIDTH, WIDTH)] * (DEPTH - 1) + [(2, WIDTH)]


def _bf16(a):
    """Round float32 to the nearest bfloat16 (ties to even), returned as float32."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def _params(seed):
    rng = np.random.default_rng(seed)
    ps = [(rng.uniform(-1, 1, s) * np.sqrt(6.0 / s[1]), rng.normal(size=s[0]) * 0.05) for s in SHAPES]
    return omlp.pack(ps).astype(np.float32)


def _inputs(rows, n, seed, bf16):
    rng = np.random.default_rng(seed)
    x = np.zeros((rows, 32), dtype=np.float32)
    x[:n, :N_IN] = rng.normal(size=(n, N_IN)).astype(np.float32)
    y = (rng.normal(size=rows) * 0.2).astype(np.float32)
    if bf16:
        x = _bf16(x)
    return x, y


def _device_x(torch, x, bf16):
    t = torch.as_tensor(x).cuda()
    return t.to(torch.bfloat16).contiguous() if bf16 else t


@pytest.mark.parametrize("mode,tol", [(1, 1e-5), (0, 2e-2)])
def test_gradients_and_heads_vs_reference(mode, tol):
    print(f"[case] mlp gradients mode={mode}", flush=True)
    torch = torch_cuda()
    import paper_2510_05100_amd as rw
    bf16 = mode == 0
    n, lam = 200, 0.3
    flat = _params(11)
    m = rw.rwgt_mlp_create(N_IN, WIDTH, DEPTH, 2, mode, 1)
    try:
        rw.rwgt_mlp_set_stream(m, None)
        rw.rwgt_mlp_set_training(m, lam)
        rw.rwgt_mlp_set_params(m, flat)
        np.testing.assert_array_equal(rw.rwgt_mlp_get_params(m), flat)
        x, y = _inputs(256, n, 5, bf16)
        xd, yd = _device_x(torch, x, bf16), torch.as_tensor(y).cuda()
        heads = torch.zeros((n, 32), dtype=torch.float32, device="cuda")
        rw.rwgt_mlp_forward(m, xd, n, heads)
        rw.rwgt_mlp_train_step(m, xd, yd, n, 0.0)
        torch.cuda.synchronize()
        grads = rw.rwgt_mlp_get_grads(m)
    finally:
        rw.rwgt_mlp_destroy(m)
    ref_params = omlp.unpack(flat.astype(np.float64), SHAPES)
    if bf16:                                   # the device multiplies with BF16 copies of the weights
        ref_params = [(_bf16(w.astype(np.float32)).astype(np.float64), b) for w, b in ref_params]
    xr = x[:n, :N_IN].astype(np.float64)
    ref_heads, _ = omlp.forward(ref_params, xr)
    got = heads.cpu().numpy()[:, :2]
    assert np.max(np.abs(got - ref_heads)) <= tol * np.max(np.abs(ref_heads)) + 1e-7
    ref_g = omlp.gradients(ref_params, xr, y[:n].astype(np.float64), lam)
    got_g = omlp.unpack(grads.astype(np.float64), SHAPES)
    for (gw, gb), (rw_, rb) in zip(got_g, ref_g):
        assert np.linalg.norm(gw - rw_) <= tol * np.linalg.norm(rw_) + 1e-12
        assert np.linalg.norm(gb - rb) <= tol * np.linalg.norm(rb) + 1e-12
    print(f"mlp mode {mode}: heads and gradients within {tol}", flush=True)


def test_features_kernel():
    print("[case] mlp features", flush=True)
    torch = torch_cuda()
    import paper_2510_05100_amd as rw
    p = synth.events("uu_eeg", 100)
    cards = np.array([[91.0, 2.5, 0.23], [90.5, 2.3, 0.22]], dtype=np.float32)
    cidx = (np.arange(100) % 2).astype(np.int32)
    mean = np.linspace(-1, 1, N_IN).astype(np.float32)
    std = np.linspace(1, 3, N_IN).astype(np.float32)
    m = rw.rwgt_mlp_create(N_IN, 64, 1, 2, 1, 0)
    try:
        rw.rwgt_mlp_set_stream(m, None)
        rw.rwgt_mlp_set_normalisation(m, mean, std)
        x = torch.zeros(rw.rwgt_mlp_input_bytes(m, 100) // 4, dtype=torch.float32, device="cuda")
        rw.rwgt_mlp_features(m, dev(p), None, torch.as_tensor(cidx).cuda(), torch.as_tensor(cards).cuda(), 100, x)
        torch.cuda.synchronize()
        got = x.cpu().numpy().reshape(-1, 32)
    finally:
        rw.rwgt_mlp_destroy(m)
    raw = np.concatenate([p.reshape(100, 20).astype(np.float32), cards[cidx]], axis=1)
    want = (raw - mean) / std
    np.testing.assert_array_equal(got[:100, :N_IN], want.astype(np.float32))
    assert np.all(got[:100, N_IN:] == 0) and np.all(got[100:] == 0)


def test_training_reduces_loss():
    print("[case] mlp training", flush=True)
    torch = torch_cuda()
    import paper_2510_05100_amd as rw
    rng = np.random.default_rng(3)
    n = 4096
    x = np.zeros((n, 32), dtype=np.float32)
    x[:, :N_IN] = rng.normal(size=(n, N_IN))
    y = (np.sin(x[:, 0]) * 0.3 + 0.1 * x[:, 1] * x[:, 2]).astype(np.float32)
    m = rw.rwgt_mlp_create(N_IN, WIDTH, DEPTH, 2, 0, 7)
    try:
        rw.rwgt_mlp_set_stream(m, None)
        rw.rwgt_mlp_set_training(m, 0.05)
        xd = torch.as_tensor(x).cuda().to(torch.bfloat16).contiguous()
        yd = torch.as_tensor(y).cuda()
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        losses = []
        for step in range(300):
            rw.rwgt_mlp_train_step(m, xd, yd, n, 2e-3, loss)
            if step % 50 == 0 or step == 299:
                torch.cuda.synchronize()
                losses.append(float(loss.item()) / n)
        heads = torch.zeros((n, 32), dtype=torch.float32, device="cuda")
        rw.rwgt_mlp_forward(m, xd, n, heads)
        torch.cuda.synchronize()
        mse = float(np.mean((heads.cpu().numpy()[:, 0] - y) ** 2))
    finally:
        rw.rwgt_mlp_destroy(m)
    print("losses", losses, "mse", mse, flush=True)
    assert mse < 0.1 * np.var(y)


def test_surrogate_path_fallback_is_exact():
    print("[case] surrogate path", flush=True)
    torch = torch_cuda()
    import paper_2510_05100_amd as rw
    n = 3000
    p = synth.events("uu_eeg", n)
    grid = synth.batch_grid()
    table = np.stack([c.row("uu_eeg") for c in grid[:8]])
    cidx = (np.arange(n) % 8).astype(np.int32)
    ctx = rw.rwgt_create(PROCESS_TEXT["uu_eeg"], synth.ORIG_EW.slha(), 0)
    m = rw.rwgt_mlp_create(N_IN, 64, 2, 2, 0, 1)
    try:
        rw.rwgt_set_stream(ctx, None)
        pd, wd = dev(p), dev(np.linspace(0.5, 2, n))
        cd = torch.as_tensor(cidx).cuda()
        exact = torch.empty(n, dtype=torch.float64, device="cuda")
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        # threshold 0: every event goes to the exact path
        nfb = rw.rwgt_sur_eval(ctx, m, pd, wd, table, cd, 0.0, exact)
        assert nfb == n
        # reference: plain rwgt_eval per card
        ref = np.empty(n)
        for k in range(8):
            sel = np.where(cidx == k)[0]
            o = torch.empty((1, sel.size), dtype=torch.float64, device="cuda")
            rw.rwgt_eval(ctx, dev(p[sel]), dev(np.linspace(0.5, 2, n)[sel]), table[k], o)
            torch.cuda.synchronize()
            ref[sel] = o.cpu().numpy()[0]
        assert np.max(rel_err(exact.cpu().numpy(), ref)) < 1e-14
        # huge threshold: no exact evaluation, w' = w exp(mu)
        nfb = rw.rwgt_sur_eval(ctx, m, pd, wd, table, cd, 1e30, out)
        assert nfb == 0
        torch.cuda.synchronize()
        assert np.all(np.isfinite(out.cpu().numpy()))
        # a threshold between: fallback events carry the exact value
        heads_thr = 3.3 * np.exp(0.0)
        nfb = rw.rwgt_sur_eval(ctx, m, pd, wd, table, cd, heads_thr, out)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        e = exact.cpu().numpy()
        same = o == e
        assert same.sum() >= nfb
        assert 0 <= nfb <= n
        # nothing to do for zero events
        assert rw.rwgt_sur_eval(ctx, m, pd[:0], wd[:0], table, cd[:0], 1e-3, out[:0]) == 0
    finally:
        rw.rwgt_mlp_destroy(m)
        rw.rwgt_destroy(ctx)


def test_surrogate_workflow_small():
    """Train on exact ratios, calibrate, evaluate with fallback (small sizes)."""
    print("[case] surrogate workflow", flush=True)
    torch = torch_cuda()
    from paper_2510_05100_amd import surrogate
    cfg = surrogate.Config(width=64, depth=2, epochs=3, batch=1024)
    summary, sur, (mean, std) = surrogate.run(torch, cfg, n_train=2000, n_heldout=20000, threshold=1e-2,
                                              log=lambda *a: print(*a, flush=True))
    try:
        assert summary["train_pairs"] == 2000 * 64
        assert summary["calibration"]["k"] > 0
        assert 0 <= summary["fallback_fraction"] <= 1
        # events the network answered are within the threshold up to the calibration coverage
        assert summary["events_beyond_threshold"] <= 0.01 * summary["heldout_events"]
    finally:
        sur.close()
