"""Pins of the oracle's Dirac algebra and external wavefunctions against the
defining equations (Dirac equation, completeness, normalisation, helicity,
transversality)."""
import numpy as np
import pytest

from oracle import lorentz as L


def _momenta(m, n=50, seed=0):
    rng = np.random.default_rng(seed)
    p3 = rng.normal(size=(n, 3)) * 300.0
    p3[0] = [0.0, 0.0, -250.0]          # exactly along -z
    p3[1] = [0.0, 0.0, 250.0]           # exactly along +z
    e = np.sqrt(m * m + np.sum(p3 ** 2, axis=1))
    return np.concatenate([e[:, None], p3], axis=1)


def test_clifford_algebra():
    g = L.GAMMA
    for mu in range(4):
        for nu in range(4):
            anti = g[mu] @ g[nu] + g[nu] @ g[mu]
            np.testing.assert_allclose(anti, 2 * L.METRIC[mu, nu] * np.eye(4), atol=1e-15)
    np.testing.assert_allclose(L.GAMMA5, 1j * g[0] @ g[1] @ g[2] @ g[3], atol=1e-15)


@pytest.mark.parametrize("m", [0.0, 173.0])
def test_dirac_equation(m):
    p = _momenta(m)
    ps = L.slash(p)
    for lam in (-1, 1):
        u = L.u_spinor(p, m, lam)
        v = L.v_spinor(p, m, lam)
        scale = p[:, 0:1]
        assert np.max(np.abs(np.einsum("nij,nj->ni", ps - m * np.eye(4), u)) / scale) < 1e-13
        assert np.max(np.abs(np.einsum("nij,nj->ni", ps + m * np.eye(4), v)) / scale) < 1e-13


@pytest.mark.parametrize("m", [0.0, 173.0])
def test_completeness_and_normalisation(m):
    p = _momenta(m)
    su = sum(np.einsum("ni,nj->nij", L.u_spinor(p, m, s), L.bar(L.u_spinor(p, m, s))) for s in (-1, 1))
    sv = sum(np.einsum("ni,nj->nij", L.v_spinor(p, m, s), L.bar(L.v_spinor(p, m, s))) for s in (-1, 1))
    scale = p[:, 0, None, None]
    assert np.max(np.abs(su - (L.slash(p) + m * np.eye(4))) / scale) < 1e-13
    assert np.max(np.abs(sv - (L.slash(p) - m * np.eye(4))) / scale) < 1e-13
    for s in (-1, 1):
        u, v = L.u_spinor(p, m, s), L.v_spinor(p, m, s)
        np.testing.assert_allclose(np.einsum("ni,ni->n", L.bar(u), u), 2 * m, atol=1e-10)
        np.testing.assert_allclose(np.einsum("ni,ni->n", L.bar(v), v), -2 * m, atol=1e-10)
        # u^dagger u = 2E
        np.testing.assert_allclose(np.sum(np.abs(u) ** 2, axis=1), 2 * p[:, 0], rtol=1e-13)


def test_helicity_eigenstates():
    p = _momenta(173.0)
    n = p[:, 1:] / np.linalg.norm(p[:, 1:], axis=1, keepdims=True)
    sig = np.einsum("ni,ijk->njk", n, L.SIGMA[1:])
    big = np.zeros((p.shape[0], 4, 4), dtype=complex)
    big[:, :2, :2] = sig
    big[:, 2:, 2:] = sig
    for lam in (-1, 1):
        u = L.u_spinor(p, 173.0, lam)
        np.testing.assert_allclose(np.einsum("nij,nj->ni", big, u), lam * u, atol=1e-10)
        # v(p, lam) describes an antiparticle of helicity lam: its spinor has spin -lam
        v = L.v_spinor(p, 173.0, lam)
        np.testing.assert_allclose(np.einsum("nij,nj->ni", big, v), -lam * v, atol=1e-10)


def test_polarisation_vectors():
    k = _momenta(0.0)
    ep, em = L.polarisation(k, 1), L.polarisation(k, -1)
    for e in (ep, em):
        np.testing.assert_allclose(L.mdot(e, k), 0, atol=1e-11)
        np.testing.assert_allclose(L.mdot(e, np.conj(e)), -1, atol=1e-14)
        np.testing.assert_allclose(e[:, 0], 0, atol=0)
    np.testing.assert_allclose(L.mdot(ep, np.conj(em)), 0, atol=1e-14)
    # helicity: (S.n) eps = lam eps with (S_k)_{ij} = -i eps_{kij}
    n = k[:, 1:] / k[:, :1]
    lc = np.zeros((3, 3, 3))
    lc[0, 1, 2] = lc[1, 2, 0] = lc[2, 0, 1] = 1
    lc[0, 2, 1] = lc[2, 1, 0] = lc[1, 0, 2] = -1
    s = -1j * lc
    sn = np.einsum("nk,kij->nij", n, s)
    for lam, e in ((1, ep), (-1, em)):
        np.testing.assert_allclose(np.einsum("nij,nj->ni", sn, e[:, 1:]), lam * e[:, 1:], atol=1e-13)
