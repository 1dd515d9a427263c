"""The stored oracle values of tests/golden/me2_oracle.json (written by
tests/golden/make_golden.py from the oracle alone): the oracle still
reproduces them (a change to its arithmetic shows up here), and they are
self-consistent (w' = |M'|^2/|M|^2 for w = 1).  The device path is compared
with them in tests/test_gpu_parity.py."""
import importlib.util
import json
import os

import numpy as np

HERE = os.path.join(os.path.dirname(__file__), "golden")


def _stored():
    with open(os.path.join(HERE, "me2_oracle.json")) as f:
        return json.load(f)


def test_oracle_reproduces_the_stored_values():
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    fresh = mod.compute()
    for a, b in zip(_stored()["cases"], fresh["cases"]):
        assert a["process"] == b["process"] and a["orig"] == b["orig"] and a["new"] == b["new"]
        for key in ("me2_orig", "me2_new", "w_new"):
            np.testing.assert_allclose(b[key], a[key], rtol=1e-12, atol=0)


def test_stored_values_are_consistent():
    for c in _stored()["cases"]:
        m0, m1, w = (np.array(c[k]) for k in ("me2_orig", "me2_new", "w_new"))
        assert np.all(m0 > 0) and np.all(m1 > 0)
        np.testing.assert_allclose(w, m1 / m0, rtol=1e-14)
        if c["process"] in ("gg_ttgg", "gg_tttt"):       # alpha_s only: (0.130/0.118)^4 on every event
            np.testing.assert_allclose(w, (0.130 / 0.118) ** 4, rtol=1e-13)
