"""g g -> t t~ + (n-2) g by colour-ordered Berends-Giele recursion, FP64.

Colour decomposition (one quark line, tree level; Mangano & Parke, Phys. Rep.
200 (1991) 301):

  M = sum_{pi in S_n} (t^{a_pi(1)} ... t^{a_pi(n)})_{i j} A(pi)

with i the colour of the outgoing top, j that of the outgoing antitop, and the
first generator of the string nearest the top.  The colour-ordered rules below
follow from the textbook QCD vertices (Peskin & Schroeder fig. 16.7: quark
vertex i g gamma^mu t^a, three-gluon vertex g f^{abc}[...], four-gluon vertex
-i g^2 [f f (...) + ...], gluon propagator -i g_{mu nu}/k^2, quark propagator
i (q-slash + m)/(q^2 - m^2)) on replacing f^{abe} t^e = -i [t^a, t^b]:

* gluon current of an ordered gluon list pi (Berends & Giele, Nucl. Phys.
  B306 (1988) 759), k_pi the summed momentum flowing in from the legs:
    J(pi) = -i/k_pi^2 [ sum_{pi = (a, b)} (-i g) V3(J_a, k_a, J_b, k_b)
                       + sum_{pi = (a, b, c)} (i g^2) V4(J_a, J_b, J_c) ]
    V3 = (J_a.J_b)(k_a - k_b) + ((k_a + 2 k_b).J_a) J_b - ((2 k_a + k_b).J_b) J_a
    V4 = 2 J_b (J_a.J_c) - J_a (J_b.J_c) - J_c (J_a.J_b)
  with J of a single leg its polarisation vector;
* off-shell antitop-side spinor, starting from v(p_tbar):
    psi(pi) = S(-p_tbar + k_pi) sum_{pi = (a, b)} (i g J_a-slash) psi(b),
    psi(()) = v(p_tbar),  S(q) = i (q-slash + m)/(q^2 - m^2);
* partial amplitude A(pi) = ubar(p_t) sum_{pi = (a, b)} (i g J_a-slash) psi(b).

Incoming gluons enter with k = +p and eps(p), outgoing ones with k = -p and
eps*(p).  |M|^2 = A_P sum_hel sum_{pi, pi'} conj(A(pi)) C[pi, pi'] A(pi') with C
from ``colour`` and A_P = 1/4 (spins) * 1/64 (colours) * 1/(n-2)! (identical
final gluons).

Pinned by: the g g -> t t~ closed form (n = 2), the Parke-Taylor MHV formula
for massless quarks, gauge invariance of every partial amplitude, Bose
symmetry, Lorentz and phase invariance, exact alpha_s^n scaling
(tests/test_oracle_gg.py).
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np

from .colour import colour_matrix, orderings
from .lorentz import bar, helicity_combinations, mdot, polarisation, slash, u_spinor, v_spinor


def v3(ja, ka, jb, kb):
    return (mdot(ja, jb)[:, None] * (ka - kb)
            + mdot(ka + 2.0 * kb, ja)[:, None] * jb
            - mdot(2.0 * ka + kb, jb)[:, None] * ja)


def v4(ja, jb, jc):
    return (2.0 * mdot(ja, jc)[:, None] * jb
            - mdot(jb, jc)[:, None] * ja
            - mdot(ja, jb)[:, None] * jc)


def partial_amplitudes(k_in, eps, ubar_t, v_tbar, p_tbar, mt, gs):
    """All n! colour-ordered amplitudes for one helicity assignment.

    k_in: [n, N, 4] gluon momenta flowing into the diagram; eps: [n, N, 4]
    their polarisation vectors; ubar_t, v_tbar: [N, 4] external spinors.
    Returns {ordering tuple: [N] complex}.
    """
    n = k_in.shape[0]
    jmemo, kmemo, pmemo = {}, {}, {}

    def mom(pi):
        if pi not in kmemo:
            kmemo[pi] = k_in[list(pi)].sum(axis=0)
        return kmemo[pi]

    def cur(pi):
        if pi in jmemo:
            return jmemo[pi]
        if len(pi) == 1:
            out = eps[pi[0]]
        else:
            acc = np.zeros_like(eps[0])
            for i in range(1, len(pi)):
                a, b = pi[:i], pi[i:]
                acc += (-1j * gs) * v3(cur(a), mom(a), cur(b), mom(b))
            for i in range(1, len(pi) - 1):
                for j in range(i + 1, len(pi)):
                    acc += (1j * gs * gs) * v4(cur(pi[:i]), cur(pi[i:j]), cur(pi[j:]))
            k = mom(pi)
            out = (-1j / mdot(k, k))[:, None] * acc
        jmemo[pi] = out
        return out

    def attach(pi):
        """sum over splits pi = (a, b) of (i g J_a-slash) psi(b)."""
        acc = np.zeros_like(v_tbar)
        for i in range(1, len(pi) + 1):
            a, b = pi[:i], pi[i:]
            acc += np.einsum("nij,nj->ni", 1j * gs * slash(cur(a)), psi(b))
        return acc

    def psi(pi):
        if pi in pmemo:
            return pmemo[pi]
        if len(pi) == 0:
            out = v_tbar
        else:
            q = -p_tbar + mom(pi)
            prop = 1j * (slash(q) + mt * np.eye(4)) / (mdot(q, q) - mt * mt)[:, None, None]
            out = np.einsum("nij,nj->ni", prop, attach(pi))
        pmemo[pi] = out
        return out

    return {pi: np.einsum("ni,ni->n", ubar_t, attach(pi)) for pi in orderings(n)}


@lru_cache(maxsize=None)
def _colour(n):
    return colour_matrix(n)


def external_states(p, hel, mt, incoming_gluons, outgoing_gluons, top, antitop):
    """Gluon (k_in, eps) and top spinors for one helicity assignment.

    ``hel`` is indexed by particle position in the event."""
    ks, es = [], []
    for i in incoming_gluons:
        ks.append(p[:, i])
        es.append(polarisation(p[:, i], hel[i]))
    for i in outgoing_gluons:
        ks.append(-p[:, i])
        es.append(np.conj(polarisation(p[:, i], hel[i])))
    ubar_t = bar(u_spinor(p[:, top], mt, hel[top]))
    v_tbar = v_spinor(p[:, antitop], mt, hel[antitop])
    return np.stack(ks), np.stack(es), ubar_t, v_tbar


def me2_ttbar_gluons(p, gs, mt, n_out_gluons):
    """|M|^2 for g(p0) g(p1) -> t(p2) t~(p3) g(p4) ... g(p_{3+n_out}).

    p: [N, 4 + n_out_gluons, 4]."""
    n = 2 + n_out_gluons
    npart = 4 + n_out_gluons
    inc, out = [0, 1], list(range(4, npart))
    cmat = _colour(n)
    perms = orderings(n)
    total = np.zeros(p.shape[0])
    for hel in helicity_combinations(npart):
        k, e, ub, v = external_states(p, hel, mt, inc, out, 2, 3)
        amps = partial_amplitudes(k, e, ub, v, p[:, 3], mt, gs)
        a = np.stack([amps[pi] for pi in perms], axis=1)        # [N, n!]
        total += np.real(np.einsum("ni,ij,nj->n", np.conj(a), cmat, a))
    average = 0.25 / 64.0 / math.factorial(n_out_gluons)
    return average * total


def me2(p: np.ndarray, card) -> np.ndarray:
    """g g -> t t~ g g: spin/colour-averaged, symmetry-factored |M|^2 per event."""
    gs = math.sqrt(4.0 * math.pi * card.aS)
    return me2_ttbar_gluons(p, gs, card.MT, 2)
