"""Helpers for the GPU tests: device tensors from synth inputs and calls
through the C ABI binding."""
import numpy as np
import pytest

PROCESS_TEXT = {"ee_mumu": "e+ e- > mu+ mu-", "uu_eeg": "u u~ > e+ e- g", "gg_ttgg": "g g > t t~ g g",
                "gg_tttt": "g g > t t~ t t~"}


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dev(x):
    torch = torch_cuda()
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def gpu_me2(process, p, orig_card, cards, precision=0):
    """|M|^2 per card from the device path, [ncards, nevt] numpy."""
    import paper_2510_05100_amd as rw
    torch = torch_cuda()
    with rw.Reweighter(PROCESS_TEXT[process], orig_card.slha(), precision) as r:
        rows = np.stack([c.row(process) for c in cards])
        out = torch.empty((len(cards), p.shape[0]), dtype=torch.float64, device="cuda")
        r.me2(dev(p), rows, out)
        torch.cuda.synchronize()
        return out.cpu().numpy()


def gpu_eval(process, p, w, orig_card, cards, precision=0):
    import paper_2510_05100_amd as rw
    torch = torch_cuda()
    with rw.Reweighter(PROCESS_TEXT[process], orig_card.slha(), precision) as r:
        rows = np.stack([c.row(process) for c in cards])
        out = torch.empty((len(cards), p.shape[0]), dtype=torch.float64, device="cuda")
        r.eval(dev(p), dev(w), rows, out)
        torch.cuda.synchronize()
        return out.cpu().numpy()


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b) / np.abs(b)
