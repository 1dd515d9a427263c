"""Surrogate training, calibration and checkpoints through the C ABI.

- rwgt_mlp_train against the same steps taken one call at a time: pairs in
  the host order of rwgt_train_order, their features (rwgt_mlp_features) and
  targets, one rwgt_mlp_train_step each at the schedule's learning rate.  The
  same kernels on the same inputs: parameters equal bit for bit, which pins
  the device shuffle to the host one, the target gather and the schedule.
- Training in two pieces with a checkpoint between them (save, destroy, load)
  against one uninterrupted run: parameters, both Adam moments and the
  progress counters equal bit for bit.
- rwgt_mlp_calibrate against the oracle's calibration quantile and order
  statistics of the same network's heads (FP64 on both sides from the same
  FP32 heads and targets): 1e-12 relative.
"""
import numpy as np
import pytest

import synth
from oracle import mlp as omlp

from gpu_util import dev, torch_cuda

pytestmark = pytest.mark.gpu

ORIG = (synth.ORIG_EW.MZ, synth.ORIG_EW.WZ)
NEVT, NCARDS = 600, 4
SCHED = dict(batch=256, epochs=4, lr=2e-3, lr_final=2e-4, seed=9)


def _grid(torch):
    p = synth.events("uu_eeg", NEVT, seed=4242)
    cards = np.stack([[c.MZ, c.WZ, c.sw2] for c in synth.batch_grid()[::16]]).astype(np.float32)
    assert cards.shape == (NCARDS, 3)
    rng = np.random.default_rng(17)
    y = (0.02 * np.log(p[:, 2, 0] / 50.0)[None, :] + 0.01 * rng.normal(size=(NCARDS, NEVT))).astype(np.float32)
    return p, cards, y, dev(p), torch.as_tensor(cards).cuda(), torch.as_tensor(y).cuda()


def _network(rw, seed=3):
    n_in = rw.n_features(rw.RWGT_FEAT_PHYS, 5)
    m = rw.rwgt_mlp_create(n_in, 128, 3, 2, rw.RWGT_MLP_BF16, seed)
    rw.rwgt_mlp_set_stream(m, None)
    rw.rwgt_mlp_set_features(m, rw.RWGT_FEAT_PHYS, 5, (2, 3), ORIG)
    rw.rwgt_mlp_set_training(m, 0.01)
    return m


def test_train_equals_manual_steps():
    print("[case] rwgt_mlp_train against manual steps", flush=True)
    torch = torch_cuda()
    import paper_2510_05100_amd as rw
    p, cards, y, pd, cd_dev, yd = _grid(torch)
    total = NEVT * NCARDS
    a, b = _network(rw), _network(rw)
    try:
        rw.rwgt_mlp_fit_grid(a, pd, cd_dev, yd)
        losses = rw.rwgt_mlp_train(a, pd, cd_dev, yd, epoch_end=SCHED["epochs"], **SCHED)
        assert losses.shape == (SCHED["epochs"],) and np.all(np.isfinite(losses))
        rw.rwgt_mlp_fit_grid(b, pd, cd_dev, yd)
        per_epoch = total // SCHED["batch"]
        nsteps = per_epoch * SCHED["epochs"]
        lr0, lr1 = float(np.float32(SCHED["lr"])), float(np.float32(SCHED["lr_final"]))
        yflat = y.reshape(-1)
        x = torch.zeros(rw.rwgt_mlp_input_bytes(b, SCHED["batch"]) // 4, dtype=torch.float32, device="cuda")
        step = 0
        for ep in range(SCHED["epochs"]):
            for k in range(per_epoch):
                j = rw.rwgt_train_order(SCHED["seed"], ep, total, k * SCHED["batch"], SCHED["batch"])
                ev = torch.as_tensor((j % NEVT).astype(np.int32)).cuda()
                cd = torch.as_tensor((j // NEVT).astype(np.int32)).cuda()
                yb = torch.as_tensor(yflat[j]).cuda()
                rw.rwgt_mlp_features(b, pd, ev, cd, cd_dev, SCHED["batch"], x)
                lr = lr0 * (lr1 / lr0) ** (step / (nsteps - 1))
                rw.rwgt_mlp_train_step(b, x, yb, SCHED["batch"], lr)
                step += 1
        torch.cuda.synchronize()
        pa, pb = rw.rwgt_mlp_get_params(a), rw.rwgt_mlp_get_params(b)
        assert rw.rwgt_mlp_get_progress(a) == (SCHED["epochs"], nsteps, nsteps)
    finally:
        rw.rwgt_mlp_destroy(a)
        rw.rwgt_mlp_destroy(b)
    np.testing.assert_array_equal(pa, pb)


def test_resume_from_checkpoint_equals_continuous(tmp_path):
    print("[case] checkpoint resume", flush=True)
    torch = torch_cuda()
    import paper_2510_05100_amd as rw
    _, _, _, pd, cd_dev, yd = _grid(torch)
    path = str(tmp_path / "sur.ckpt")
    a, b, c = _network(rw), _network(rw), None
    try:
        rw.rwgt_mlp_fit_grid(a, pd, cd_dev, yd)
        rw.rwgt_mlp_train(a, pd, cd_dev, yd, epoch_end=4, **SCHED)
        rw.rwgt_mlp_fit_grid(b, pd, cd_dev, yd)
        rw.rwgt_mlp_train(b, pd, cd_dev, yd, epoch_end=2, **SCHED)
        rw.rwgt_mlp_set_calibration(b, 2.5)
        rw.rwgt_mlp_save(b, path)
        before = rw.rwgt_mlp_get_params(b)
        rw.rwgt_mlp_destroy(b)
        b = None
        shape, epoch, steps = rw.rwgt_mlp_checkpoint_info(path)
        assert shape == (18, 128, 3, 2, rw.RWGT_MLP_BF16) and epoch == 2 and steps == 2 * (2400 // 256)
        c = rw.rwgt_mlp_load(path)
        rw.rwgt_mlp_set_stream(c, None)
        np.testing.assert_array_equal(rw.rwgt_mlp_get_params(c), before)
        # a changed schedule is refused
        bad = dict(SCHED, lr=1e-3)
        with pytest.raises(rw.RwgtError, match="schedule"):
            rw.rwgt_mlp_train(c, pd, cd_dev, yd, epoch_end=4, **bad)
        rw.rwgt_mlp_train(c, pd, cd_dev, yd, epoch_end=4, **SCHED)
        torch.cuda.synchronize()
        assert rw.rwgt_mlp_get_progress(c) == rw.rwgt_mlp_get_progress(a)
        np.testing.assert_array_equal(rw.rwgt_mlp_get_params(c), rw.rwgt_mlp_get_params(a))
        ma, va, ta = rw.rwgt_mlp_get_adam(a)
        mc, vc, tc = rw.rwgt_mlp_get_adam(c)
        assert ta == tc
        np.testing.assert_array_equal(ma, mc)
        np.testing.assert_array_equal(va, vc)
        # the loaded network predicts with the saved normalisation and scale
        mean_a, std_a, ys_a = rw.rwgt_mlp_get_normalisation(a, 18)
        mean_c, std_c, ys_c = rw.rwgt_mlp_get_normalisation(c, 18)
        np.testing.assert_array_equal(mean_a, mean_c)
        np.testing.assert_array_equal(std_a, std_c)
        assert tuple(ys_a) == tuple(ys_c)
    finally:
        for m in (a, b, c):
            if m:
                rw.rwgt_mlp_destroy(m)


def test_calibrate_vs_oracle():
    print("[case] calibration quantile", flush=True)
    torch = torch_cuda()
    import paper_2510_05100_amd as rw
    _, _, y, pd, cd_dev, yd = _grid(torch)
    total = NEVT * NCARDS
    m = _network(rw)
    try:
        rw.rwgt_mlp_fit_grid(m, pd, cd_dev, yd)
        rw.rwgt_mlp_train(m, pd, cd_dev, yd, epoch_end=2, **SCHED)
        stats = rw.rwgt_mlp_calibrate(m, pd, cd_dev, yd, 0.99)
        j = np.arange(total)
        heads = torch.empty((total, 2), dtype=torch.float32, device="cuda")
        rw.rwgt_mlp_predict(m, pd, torch.as_tensor((j % NEVT).astype(np.int32)).cuda(),
                            torch.as_tensor((j // NEVT).astype(np.int32)).cuda(), cd_dev, total, heads)
        torch.cuda.synchronize()
        h = heads.cpu().numpy().astype(np.float64)
    finally:
        rw.rwgt_mlp_destroy(m)
    yy = y.reshape(-1).astype(np.float64)
    k = omlp.calibration_k(yy, h[:, 0], h[:, 1], 0.99)
    r = np.abs(yy - h[:, 0])
    want = (k, omlp.quantile_linear(r, 0.5), omlp.quantile_linear(r, 0.9), omlp.quantile_linear(r, 0.999))
    print("calibration", stats, "oracle", want, flush=True)
    np.testing.assert_allclose(stats, want, rtol=1e-12)
    with pytest.raises(rw.RwgtError, match="coverage"):
        m2 = _network(rw)
        try:
            rw.rwgt_mlp_calibrate(m2, pd, cd_dev, yd, 1.0)
        finally:
            rw.rwgt_mlp_destroy(m2)
