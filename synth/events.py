"""Synthetic LHCb-like events: primary vertices and the VELO tracks they emit.

The paper measures on LHCb Run-3 simulation (5.6 primary vertices per event on
average, Section 1), which is not available here; this generator stands in for
it.  Per event, in this draw order, from the ``events`` stream:

1. ``n_pv ~ Poisson(5.6)``, redrawn while it is 0.
2. Track count ``T``: ``Poisson(180)`` ("poisson" mix) or
   ``clip(round(LogNormal(ln 180, sigma)), 5, 1500)`` ("lognormal" mix, the
   heavy-tailed batches).
3. PV ``z ~ N(0, 45 mm)`` clipped to [-100, 300] mm, then PV ``x``, ``y`` each
   ``~ N(0, 0.04 mm)``.
4. Track-to-PV counts ``~ Multinomial(T, uniform over the PVs)``; the track list
   is then shuffled with one permutation.
5. Track features: ``z = PVz + N(0, 0.1)``, ``x = PVx + N(0, 0.05)``,
   ``y = PVy + N(0, 0.05)``, three covariance terms ``exp(N(-3, 0.5))``, three
   slope/momentum terms ``N(0, 0.2)``.  Drawn in float64, stored as float32.

Track z is not clipped, so tracks of a PV near -100 mm can fall outside the
histogram window; the method drops those.

Layout (structure of arrays, as the trigger framework stores tracks): one
float32 plane per feature, ``feat[9][T_total]``, events back to back, and
``offsets[E+1]`` (int32) with event ``e`` owning tracks
``offsets[e] .. offsets[e+1]-1``.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Feature order inside one track record.
TRACK_FEATURES = ("z", "x", "y", "c1", "c2", "c3", "s1", "s2", "s3")
N_FEAT = len(TRACK_FEATURES)

MEAN_PV = 5.6
MEAN_TRACKS = 180.0
PV_Z_SIGMA = 45.0
PV_Z_LO, PV_Z_HI = -100.0, 300.0
PV_XY_SIGMA = 0.04
TRK_Z_SIGMA = 0.1
TRK_XY_SIGMA = 0.05
COV_MU, COV_SIGMA = -3.0, 0.5
SLOPE_SIGMA = 0.2
LOGNORMAL_SIGMA = 1.0
T_MIN, T_MAX = 5, 1500


@dataclass
class EventBatch:
    feat: np.ndarray            # float32 [9][T_total], SoA planes
    offsets: np.ndarray         # int32 [E+1]
    pv_z: list = field(default_factory=list)   # per event: float64 true PV z (mm)

    @property
    def n_events(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_tracks_total(self) -> int:
        return int(self.offsets[-1])

    def tracks_of(self, e: int) -> np.ndarray:
        """float32 [9][T_e] view of event e's tracks."""
        return self.feat[:, self.offsets[e]:self.offsets[e + 1]]

    def subset(self, idx) -> "EventBatch":
        """A new batch holding the listed events, in the listed order."""
        idx = list(idx)
        counts = [int(self.offsets[e + 1] - self.offsets[e]) for e in idx]
        off = np.zeros(len(idx) + 1, dtype=np.int32)
        off[1:] = np.cumsum(counts)
        feat = np.empty((N_FEAT, int(off[-1])), dtype=np.float32)
        for k, e in enumerate(idx):
            feat[:, off[k]:off[k + 1]] = self.tracks_of(e)
        return EventBatch(feat, off, [self.pv_z[e] for e in idx] if self.pv_z else [])


def _events_rng(seed: int) -> np.random.Generator:
    _, ev_ss = np.random.SeedSequence(seed).spawn(2)
    return np.random.Generator(np.random.PCG64(ev_ss))


def _draw_event(rng: np.random.Generator, mix: str):
    n_pv = 0
    while n_pv == 0:
        n_pv = int(rng.poisson(MEAN_PV))
    if mix == "poisson":
        T = int(rng.poisson(MEAN_TRACKS))
    elif mix == "lognormal":
        T = int(np.clip(np.rint(rng.lognormal(np.log(MEAN_TRACKS), LOGNORMAL_SIGMA)), T_MIN, T_MAX))
    else:
        raise ValueError(f"unknown track-count mix {mix!r}")
    pv_z = np.clip(rng.normal(0.0, PV_Z_SIGMA, n_pv), PV_Z_LO, PV_Z_HI)
    pv_x = rng.normal(0.0, PV_XY_SIGMA, n_pv)
    pv_y = rng.normal(0.0, PV_XY_SIGMA, n_pv)
    counts = rng.multinomial(T, np.full(n_pv, 1.0 / n_pv))
    owner = np.repeat(np.arange(n_pv), counts)
    owner = owner[rng.permutation(T)]
    f = np.empty((N_FEAT, T), dtype=np.float64)
    f[0] = pv_z[owner] + rng.normal(0.0, TRK_Z_SIGMA, T)
    f[1] = pv_x[owner] + rng.normal(0.0, TRK_XY_SIGMA, T)
    f[2] = pv_y[owner] + rng.normal(0.0, TRK_XY_SIGMA, T)
    f[3:6] = np.exp(rng.normal(COV_MU, COV_SIGMA, (3, T)))
    f[6:9] = rng.normal(0.0, SLOPE_SIGMA, (3, T))
    return f.astype(np.float32), pv_z


def make_events(n_events: int, seed: int = 0, mix: str = "poisson") -> EventBatch:
    """Draw ``n_events`` events from the ``events`` stream of ``seed``."""
    if n_events < 0:
        raise ValueError("n_events must be >= 0")
    rng = _events_rng(seed)
    planes, truth = [], []
    off = np.zeros(n_events + 1, dtype=np.int64)
    for e in range(n_events):
        f, pvz = _draw_event(rng, mix)
        planes.append(f)
        truth.append(pvz)
        off[e + 1] = off[e] + f.shape[1]
    if off[-1] > np.iinfo(np.int32).max:
        raise ValueError("track total exceeds int32 offsets")
    feat = np.concatenate(planes, axis=1) if planes else np.zeros((N_FEAT, 0), np.float32)
    return EventBatch(np.ascontiguousarray(feat, dtype=np.float32), off.astype(np.int32), truth)


def pack_events(track_lists) -> EventBatch:
    """Build a batch from explicit per-event float32 [9][T_e] arrays (hand-made cases)."""
    counts = [int(np.asarray(t).shape[1]) for t in track_lists]
    off = np.zeros(len(counts) + 1, dtype=np.int32)
    off[1:] = np.cumsum(counts)
    feat = np.zeros((N_FEAT, int(off[-1])), dtype=np.float32)
    for e, t in enumerate(track_lists):
        feat[:, off[e]:off[e + 1]] = np.asarray(t, dtype=np.float32)
    return EventBatch(feat, off, [])
