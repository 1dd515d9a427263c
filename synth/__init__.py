"""Seeded synthetic inputs (phase-space points, weights and parameter cards).

Shared by the oracle-side tests and the device-side tests and benchmark; holds
no matrix-element arithmetic.
"""
from .rambo import massless_weight, rambo_massive, rambo_massless  # noqa: F401
from .workloads import (  # noqa: F401
    Card, GENERATORS, NEW_EE, NEW_QCD, NEW_UU, ORIG_EW, ORIG_QCD, PARAM_LAYOUT,
    PROCESSES, batch_counts, batch_grid, delta_r, events, pt, rapidity, surrogate_cards,
)
