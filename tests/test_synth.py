"""Input generators: RAMBO invariants, cuts, seeding (no matrix elements)."""
import math

import numpy as np

import synth
from synth import workloads as wl


def _mdot(a, b):
    return a[..., 0] * b[..., 0] - np.sum(a[..., 1:] * b[..., 1:], axis=-1)


def test_rambo_massless_conservation_and_shell():
    rng = np.random.default_rng(1)
    roots = rng.uniform(100, 1000, 500)
    p = synth.rambo_massless(rng, 500, 5, roots)
    tot = p.sum(axis=1)
    np.testing.assert_allclose(tot[:, 0], roots, rtol=1e-13)
    assert np.max(np.abs(tot[:, 1:]) / roots[:, None]) < 1e-13
    assert np.max(np.abs(_mdot(p, p)) / roots[:, None] ** 2) < 1e-12


def test_rambo_massive_conservation_and_shell():
    rng = np.random.default_rng(2)
    masses = np.array([173.0, 173.0, 0.0, 0.0])
    roots = rng.uniform(500, 2000, 400)
    p = synth.rambo_massive(rng, 400, masses, roots)
    tot = p.sum(axis=1)
    np.testing.assert_allclose(tot[:, 0], roots, rtol=1e-12)
    assert np.max(np.abs(tot[:, 1:]) / roots[:, None]) < 1e-12
    m2 = _mdot(p, p)
    np.testing.assert_allclose(m2, np.broadcast_to(masses ** 2, m2.shape), atol=1e-7 * 2000 ** 2)


def test_massless_phase_space_volume():
    # two-body: 4 pi * |p|^2/(2E 2E) * dE/d|p| ... = pi/2; three-body: pi^2 s / 8
    assert math.isclose(synth.massless_weight(2, 1.0), math.pi / 2, rel_tol=1e-15)
    s = 640000.0
    assert math.isclose(synth.massless_weight(3, s), math.pi ** 2 * s / 8, rel_tol=1e-15)
    # with the (2 pi)^(4 - 3n) factors the 3-body volume is s / (256 pi^3)
    assert math.isclose(synth.massless_weight(3, s) * (2 * math.pi) ** (4 - 9), s / (256 * math.pi ** 3),
                        rel_tol=1e-14)


def test_rambo_isotropic_two_body():
    # RAMBO's two-body point is isotropic: <cos theta> ~ 0, <cos^2 theta> ~ 1/3
    rng = np.random.default_rng(3)
    p = synth.rambo_massless(rng, 200000, 2, np.full(200000, 100.0))
    c = p[:, 0, 3] / p[:, 0, 0]
    assert abs(c.mean()) < 0.01
    assert abs((c ** 2).mean() - 1 / 3) < 0.01


def test_workload_cuts_and_order():
    p = synth.events("uu_eeg", 3000)
    assert p.shape == (3000, 5, 4)
    assert np.all(synth.pt(p[:, 4]) > 20.0)
    assert np.all(synth.delta_r(p[:, 4], p[:, 2]) > 0.4)
    assert np.all(synth.delta_r(p[:, 4], p[:, 3]) > 0.4)
    tot = p[:, 0] + p[:, 1] - p[:, 2:].sum(axis=1)
    assert np.max(np.abs(tot)) < 1e-9
    roots = 2 * p[:, 0, 0]
    assert roots.min() >= 150.0 and roots.max() <= 1000.0

    q = synth.events("gg_ttgg", 2000)
    assert q.shape == (2000, 6, 4)
    assert np.all(synth.pt(q[:, 4]) > 30.0) and np.all(synth.pt(q[:, 5]) > 30.0)
    assert np.all(synth.delta_r(q[:, 4], q[:, 5]) > 0.4)
    np.testing.assert_allclose(_mdot(q[:, 2], q[:, 2]), 173.0 ** 2, rtol=1e-9)


def test_ee_kinematics():
    p = synth.events("ee_mumu", 1000)
    assert np.allclose(p[:, 0], [100, 0, 0, 100]) and np.allclose(p[:, 1], [100, 0, 0, -100])
    np.testing.assert_allclose(p[:, 2] + p[:, 3], p[:, 0] + p[:, 1], atol=1e-12)


def test_seed_reproducible_and_prefix_stable():
    a = synth.events("gg_ttgg", 500)
    b = synth.events("gg_ttgg", 1200)
    np.testing.assert_array_equal(a, b[:500])
    c = synth.events("ee_mumu", 10)
    d = synth.events("ee_mumu", 100)
    np.testing.assert_array_equal(c, d[:10])
    e = synth.events("gg_ttgg", 50, seed=99)
    assert not np.array_equal(e, a[:50])


def test_batch_grid_and_counts():
    grid = synth.batch_grid()
    assert len(grid) == 64
    assert {c.MZ for c in grid} == {90.5, 91.0, 91.5, 92.0}
    assert min(c.WZ for c in grid) == 2.3 and max(c.WZ for c in grid) == 2.7
    counts = synth.batch_counts()
    assert counts.shape == (64, 2)
    assert counts.min() >= 1000 and counts.max() <= 200000
    np.testing.assert_array_equal(counts, synth.batch_counts())


def test_card_rows_and_slha():
    row = synth.NEW_UU.row("uu_eeg")
    np.testing.assert_array_equal(row, [132.507, 0.118, 0.2312, 91.5, 2.6])
    text = synth.ORIG_QCD.slha()
    assert "BLOCK SMINPUTS" in text and "3 0.118" in text
    assert wl.PARAM_LAYOUT["gg_ttgg"] == ("SMINPUTS 3", "MASS 6")
