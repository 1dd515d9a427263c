"""Reweighted cross section and its error (paper, teaRex section), FP64.

  sigma' = C sum_i w'_i
  dsigma' = dsigma * (1/N) sum_i w'_i / w_i + sigma * std(w')

std is the population standard deviation (a reading: the paper says "the
standard deviation of a variable"); terms with w_i = 0 count as 0 (a reading:
their w'_i is 0 by the 1/0 -> 0 normaliser guard).  If dsigma' is infinite,
NaN or not positive, it is replaced by dsigma times the larger of
sigma'/sigma and sigma/sigma' (the paper's conservative fallback).

Pinned by hand-computed cases (tests/test_oracle_xsec.py).
"""
from __future__ import annotations

import numpy as np


def xsec(w_in, w_out, sigma, dsigma, norm):
    w_in = np.asarray(w_in, dtype=np.float64)
    w_out = np.atleast_2d(np.asarray(w_out, dtype=np.float64))
    n = w_in.size
    xs = norm * w_out.sum(axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(w_in != 0.0, w_out / np.where(w_in != 0.0, w_in, 1.0), 0.0)
    err = dsigma * ratio.sum(axis=1) / n + sigma * w_out.std(axis=1)
    bad = ~np.isfinite(err) | ~(err > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        alt = dsigma * np.maximum(xs / sigma, sigma / xs)
    err = np.where(bad, alt, err)
    return xs, err, bad
