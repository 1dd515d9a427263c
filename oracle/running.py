"""Running strong coupling at one loop (test infrastructure).

alpha_s(mu) = alpha_s(M) / (1 + alpha_s(M) b0 ln(mu^2 / M^2)),
b0 = (33 - 2 n_f) / (12 pi), from the reference scale M = 91.1876 GeV with
n_f = 5 (readings: the paper prints no running; these are the textbook
one-loop solution and the usual reference scale).  Pinned by the value at the
reference scale, the renormalisation-group equation
d alpha / d ln mu^2 = -b0 alpha^2 (finite differences) and the composition
law of the one-loop solution (tests/test_oracle_running.py).
"""
from __future__ import annotations

import numpy as np

MZ_REF = 91.1876
NF = 5


def b0(nf=NF):
    return (33.0 - 2.0 * nf) / (12.0 * np.pi)


def alphas(as_ref, mu, mu_ref=MZ_REF, nf=NF):
    mu = np.asarray(mu, dtype=np.float64)
    return as_ref / (1.0 + as_ref * b0(nf) * np.log(mu * mu / (mu_ref * mu_ref)))
