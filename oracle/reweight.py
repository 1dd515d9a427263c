"""Reweighting result per event, FP64 (paper: teaRex section).

For event weights w and the original card theta, each new card theta_k gives

  norm_i = w_i * (1/|M|^2(p_i; theta))   with 1/0 -> 0   (teaRex section: normalisation)
  w'_ki  = norm_i * |M|^2(p_i; theta_k)                  (teaRex section: new weights)

i.e. w' = w |M'|^2/|M|^2 (the parameter-reweighting ratio of the teaRex
introduction), evaluated in that order.  The cross section and its error
(sigma' = C sum_i w'_i and the Gaussian propagation of the same section) are
in ``xsec``.
"""
from __future__ import annotations

import numpy as np

from . import ee_mumu, qcd_bg, qcd_dressed, uu_eeg

ME2 = {"ee_mumu": ee_mumu.me2, "uu_eeg": uu_eeg.me2, "gg_ttgg": qcd_bg.me2, "gg_tttt": qcd_dressed.me2_gg_tttt}


def me2(process: str, p: np.ndarray, card) -> np.ndarray:
    return ME2[process](np.asarray(p, dtype=np.float64), card)


def normalisation(w, me2_orig):
    w = np.asarray(w, dtype=np.float64)
    inv = np.zeros_like(me2_orig)
    nz = me2_orig != 0.0
    inv[nz] = 1.0 / me2_orig[nz]
    return w * inv


def reweight(process: str, p, w, card_orig, cards_new):
    """w'[k, i] for each new card k; returns (w', |M|^2 original, |M|^2 new)."""
    m0 = me2(process, p, card_orig)
    norm = normalisation(w, m0)
    mk = np.stack([me2(process, p, c) for c in cards_new])
    return norm[None, :] * mk, m0, mk
