"""The process compiler's generated amplitude code, instantiated on the host in
double precision (tests/host/generated_me.cpp), against the oracle: the same
source the device kernels instantiate, checked without a GPU.  Both QCD
processes: g g -> t t~ g g (one coloured line) against the colour-ordered
recursion, g g -> t t~ t t~ (two coloured lines: pairings with the Fermi sign,
the Fierz-reduced two-string colour basis) against the colour-dressed
recursion; 1e-12 relative (different algorithms in double).

Helicity reversal: for both (pure QCD) the generated header lists one
helicity of each reversed pair first (NSUM = 32 of 64, weight HELW = 2), and
the kernels evaluate only those.  Checked here per helicity: every reversed
pair has equal |M_h|^2 (1e-14 of the event's sum; the generated code gives
them bit for bit), the first NSUM are one of each pair, and their sum times 2
equals the full sum.  That the relation is physics, and not a property of the
generated code alone, is pinned on the oracle (tests/test_oracle_dressed.py).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth
from oracle import reweight

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_05100_amd", "csrc")


def _hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        pytest.skip("hipcc not available")
    return exe


def _build(tmp_path, name):
    exe = str(tmp_path / f"me_{name}")
    cmd = [_hipcc(), "-O1", "-std=c++17", "-I" + CSRC, f'-DGEN_HEADER="generated/gen_{name}.h"',
           f"-DGEN_NS=gen_{name}", os.path.join(ROOT, "tests", "host", "generated_me.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def _run(exe, p, card, *args):
    text = f"{p.shape[0]} {card.aS!r} {card.MT!r}\n" + "\n".join(
        " ".join("%.17g" % x for x in ev.reshape(-1)) for ev in p)
    r = subprocess.run([exe, *args], input=text, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return np.array([float(x) for x in r.stdout.split()])


@pytest.mark.parametrize("name,n", [("gg_ttgg", 6), ("gg_tttt", 4)])
def test_generated_code_on_host_against_oracle(tmp_path, name, n):
    exe = _build(tmp_path, name)
    p = synth.events(name, 50)[np.linspace(0, 49, n).astype(int)]
    got = _run(exe, p, synth.ORIG_QCD)
    want = reweight.me2(name, p, synth.ORIG_QCD)
    np.testing.assert_allclose(got, want, rtol=1e-12)


@pytest.mark.parametrize("name", ["gg_ttgg", "gg_tttt"])
def test_reversed_helicities_equal(tmp_path, name):
    exe = _build(tmp_path, name)
    n = 25
    p = synth.events(name, 200, seed=77)[::8][:n]
    out = _run(exe, p, synth.ORIG_QCD, "hel")
    ngood, nsum, helw = int(out[0]), int(out[1]), out[2]
    assert (ngood, nsum, helw) == (64, 32, 2.0)
    rec = out[3:].reshape(n, ngood, 2)
    hel = rec[0, :, 0].astype(int)
    full = 63
    assert sorted(hel) == list(range(64))
    first = set(hel[:nsum])
    assert all((full ^ h) not in first for h in first)     # one of each reversed pair
    for e in range(n):
        mh = dict(zip(rec[e, :, 0].astype(int), rec[e, :, 1]))
        tot = sum(mh.values())
        assert tot > 0
        assert max(abs(mh[h] - mh[full ^ h]) for h in mh) <= 1e-14 * tot
        half = sum(mh[h] for h in hel[:nsum])
        assert abs(helw * half - tot) <= 1e-14 * tot
