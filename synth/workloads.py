"""Seeded synthetic workloads: momenta, input weights and parameter cards.

Every function here draws from ``numpy.random.default_rng(seed)`` and returns
plain arrays, so that the oracle-side tests and the device-side tests and
benchmark see byte-identical inputs.  The module holds none of the
matrix-element arithmetic.

Particle order inside each event is the order of the process string, incoming
first; momenta are (E, px, py, pz) in GeV in the partonic centre-of-mass frame.
Candidates are drawn in fixed-size chunks, so the first n accepted events are
the same whatever total is asked for.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .rambo import rambo_massive, rambo_massless

PROCESSES = {
    "ee_mumu": "e+ e- > mu+ mu-",
    "uu_eeg": "u u~ > e+ e- g",
    "gg_ttgg": "g g > t t~ g g",
    "gg_tttt": "g g > t t~ t t~",
}

# Names of the per-card parameters each process depends on, in the order of a
# row of ``param_sets`` (SLHA block and index; RWGTEW 1 is sin^2(theta_W)).
PARAM_LAYOUT = {
    "ee_mumu": ("SMINPUTS 1", "RWGTEW 1", "MASS 23", "DECAY 23"),
    "uu_eeg": ("SMINPUTS 1", "SMINPUTS 3", "RWGTEW 1", "MASS 23", "DECAY 23"),
    "gg_ttgg": ("SMINPUTS 3", "MASS 6"),
    "gg_tttt": ("SMINPUTS 3", "MASS 6"),
}

CHUNK = 1 << 16


@dataclasses.dataclass(frozen=True)
class Card:
    """One parameter card: 1/alpha, alpha_s, sin^2(theta_W), M_Z, Gamma_Z, m_t."""
    aEWM1: float = 132.507
    aS: float = 0.118
    sw2: float = 0.2222
    MZ: float = 91.188
    WZ: float = 2.441
    MT: float = 173.0

    def value(self, name: str) -> float:
        return {
            "SMINPUTS 1": self.aEWM1, "SMINPUTS 3": self.aS, "RWGTEW 1": self.sw2,
            "MASS 23": self.MZ, "DECAY 23": self.WZ, "MASS 6": self.MT,
        }[name]

    def row(self, process: str) -> np.ndarray:
        return np.array([self.value(n) for n in PARAM_LAYOUT[process]], dtype=np.float64)

    def slha(self) -> str:
        """SLHA text of the card (only the entries these processes read)."""
        return (
            "BLOCK SMINPUTS\n"
            f"    1 {self.aEWM1!r} # aEWM1\n"
            f"    3 {self.aS!r} # aS\n"
            "BLOCK RWGTEW\n"
            f"    1 {self.sw2!r} # sw2\n"
            "BLOCK MASS\n"
            f"    6 {self.MT!r} # MT\n"
            f"   23 {self.MZ!r} # MZ\n"
            f"DECAY 23 {self.WZ!r} # WZ\n"
            "DECAY 6 0.0 # WT\n"
        )


ORIG_EW = Card()
NEW_EE = dataclasses.replace(ORIG_EW, MZ=91.5, WZ=2.6)
NEW_UU = dataclasses.replace(ORIG_EW, MZ=91.5, WZ=2.6, sw2=0.2312)
ORIG_QCD = Card(aS=0.118, MT=173.0)
NEW_QCD = dataclasses.replace(ORIG_QCD, aS=0.130)

SEED_EVENTS = {"ee_mumu": 1000, "uu_eeg": 1001, "gg_ttgg": 1002, "gg_tttt": 1003}
SEED_BATCH_COUNTS = 2000
SEED_SUR_TRAIN = 3000
SEED_SUR_HELDOUT = 3001
SEED_SUR_CARDS = 3101


# ---------------------------------------------------------------- observables
def pt(p):
    return np.hypot(p[..., 1], p[..., 2])


def rapidity(p):
    return 0.5 * np.log((p[..., 0] + p[..., 3]) / (p[..., 0] - p[..., 3]))


def delta_r(a, b):
    dphi = np.arctan2(a[..., 2], a[..., 1]) - np.arctan2(b[..., 2], b[..., 1])
    dphi = (dphi + math.pi) % (2.0 * math.pi) - math.pi
    return np.hypot(rapidity(a) - rapidity(b), dphi)


def _beams(sqrt_s):
    n = sqrt_s.shape[0]
    half = 0.5 * sqrt_s
    b = np.zeros((n, 2, 4))
    b[:, 0, 0] = half
    b[:, 0, 3] = half
    b[:, 1, 0] = half
    b[:, 1, 3] = -half
    return b


# ---------------------------------------------------------------- generators
def ee_mumu_events(n: int, seed: int = SEED_EVENTS["ee_mumu"], sqrt_s: float = 200.0) -> np.ndarray:
    """e+ (along +z) e- (along -z) -> mu+ (along n(theta, phi)) mu- (opposite);
    cos(theta) uniform in [-1, 1], phi uniform in [0, 2 pi)."""
    rng = np.random.default_rng(seed)
    r = rng.random((n, 2))
    cos_t = 2.0 * r[:, 0] - 1.0
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t ** 2))
    phi = 2.0 * math.pi * r[:, 1]
    e = 0.5 * sqrt_s
    p = np.zeros((n, 4, 4))
    p[:, :2] = _beams(np.full(n, sqrt_s))
    nvec = np.stack([sin_t * np.cos(phi), sin_t * np.sin(phi), cos_t], axis=1)
    p[:, 2, 0] = e
    p[:, 2, 1:] = e * nvec
    p[:, 3, 0] = e
    p[:, 3, 1:] = -e * nvec
    return p


def uu_eeg_events(n: int, seed: int = SEED_EVENTS["uu_eeg"]) -> np.ndarray:
    """u (+z) u~ (-z) -> e+ e- g; sqrt(s_hat) uniform in [150, 1000] GeV,
    massless 3-body RAMBO; accepted if pT(g) > 20 GeV and dR(g, e+-) > 0.4."""
    rng = np.random.default_rng(seed)
    out = []
    have = 0
    while have < n:
        sqrt_s = rng.uniform(150.0, 1000.0, CHUNK)
        fin = rambo_massless(rng, CHUNK, 3, sqrt_s)
        g, ep, em = fin[:, 2], fin[:, 0], fin[:, 1]
        ok = (pt(g) > 20.0) & (delta_r(g, ep) > 0.4) & (delta_r(g, em) > 0.4)
        ev = np.concatenate([_beams(sqrt_s), fin], axis=1)[ok]
        out.append(ev)
        have += ev.shape[0]
    return np.concatenate(out)[:n]


def gg_ttgg_events(n: int, seed: int = SEED_EVENTS["gg_ttgg"], mt: float = 173.0) -> np.ndarray:
    """g (+z) g (-z) -> t t~ g g; sqrt(s_hat) uniform in [500, 2000] GeV,
    massive 4-body RAMBO (mt, mt, 0, 0); accepted if both gluons have
    pT > 30 GeV and dR(g, g) > 0.4."""
    rng = np.random.default_rng(seed)
    out = []
    have = 0
    while have < n:
        sqrt_s = rng.uniform(500.0, 2000.0, CHUNK)
        fin = rambo_massive(rng, CHUNK, [mt, mt, 0.0, 0.0], sqrt_s)
        g1, g2 = fin[:, 2], fin[:, 3]
        ok = (pt(g1) > 30.0) & (pt(g2) > 30.0) & (delta_r(g1, g2) > 0.4)
        ev = np.concatenate([_beams(sqrt_s), fin], axis=1)[ok]
        out.append(ev)
        have += ev.shape[0]
    return np.concatenate(out)[:n]


def gg_tttt_events(n: int, seed: int = SEED_EVENTS["gg_tttt"], mt: float = 173.0) -> np.ndarray:
    """g (+z) g (-z) -> t t~ t t~; sqrt(s_hat) uniform in [800, 2500] GeV,
    massive 4-body RAMBO (four times mt); no cuts (every final particle is
    massive)."""
    rng = np.random.default_rng(seed)
    sqrt_s = rng.uniform(800.0, 2500.0, n)
    fin = rambo_massive(rng, n, [mt, mt, mt, mt], sqrt_s)
    return np.concatenate([_beams(sqrt_s), fin], axis=1)


GENERATORS = {"ee_mumu": ee_mumu_events, "uu_eeg": uu_eeg_events, "gg_ttgg": gg_ttgg_events,
              "gg_tttt": gg_tttt_events}


def events(process: str, n: int, seed: int | None = None) -> np.ndarray:
    gen = GENERATORS[process]
    return gen(n) if seed is None else gen(n, seed)


# ------------------------------------------------------ batched multi-card mix
def batch_grid():
    """4 x 4 x 4 grid of cards (M_Z, Gamma_Z, sin^2 theta_W), endpoints included,
    M_Z slowest and sin^2 theta_W fastest."""
    cards = []
    for mz in np.linspace(90.5, 92.0, 4):
        for wz in np.linspace(2.3, 2.7, 4):
            for sw2 in np.linspace(0.220, 0.235, 4):
                cards.append(dataclasses.replace(ORIG_EW, MZ=float(mz), WZ=float(wz), sw2=float(sw2)))
    return cards


def batch_counts(seed: int = SEED_BATCH_COUNTS, lo: float = 1e3, hi: float = 2e5) -> np.ndarray:
    """Per (card, process) event counts, log-uniform in [lo, hi]; shape [64, 2]
    with column 0 for e+e- -> mu+mu- and column 1 for u u~ -> e+e- g."""
    rng = np.random.default_rng(seed)
    u = rng.random((64, 2))
    return np.rint(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)


def surrogate_cards(n: int, seed: int = SEED_SUR_CARDS) -> np.ndarray:
    """Index into ``batch_grid()`` drawn uniformly per held-out event."""
    return np.random.default_rng(seed).integers(0, 64, n)
