"""Pins of the oracle's FC stage + histogram (Section 2: every track's FC output
is combined into the event histogram; Section 3: one track feeds the interval
that holds it).  The properties below hold for the exact sum whatever the
order of the tracks."""

import numpy as np
import pytest

import oracle
from synth import make_events, make_weights
from synth.events import pack_events
from tests import torch_ref

W = make_weights(0)
GEO = oracle.Geometry()


def _event(e=0, n=4):
    return make_events(n, seed=0).tracks_of(e)


def test_histogram_vs_torch_restatement():
    ev = make_events(4, seed=0)
    for e in range(4):
        H, d = oracle.histogram(ev.tracks_of(e), W, GEO)
        ref = torch_ref.histogram(ev.tracks_of(e), W).numpy()
        np.testing.assert_allclose(H, ref, rtol=1e-12, atol=0)
        assert np.array_equal(H == 0, ref == 0)


def test_track_order_invariance():
    tr = _event(1)
    H, _ = oracle.histogram(tr, W, GEO)
    perm = np.random.default_rng(5).permutation(tr.shape[1])
    Hp, _ = oracle.histogram(tr[:, perm], W, GEO)
    np.testing.assert_allclose(Hp, H, rtol=1e-13, atol=0)


def test_linearity_over_track_sets():
    tr = _event(2)
    a, b = tr[:, :70], tr[:, 70:]
    H, _ = oracle.histogram(tr, W, GEO)
    Ha, _ = oracle.histogram(a, W, GEO)
    Hb, _ = oracle.histogram(b, W, GEO)
    np.testing.assert_allclose(Ha + Hb, H, rtol=1e-13, atol=0)


def test_single_track_fills_its_interval_only():
    tr = _event(0)[:, 5:6].copy()
    tr[0, 0] = np.float32(12.34)               # interval 11: [10, 20) mm
    H, d = oracle.histogram(tr, W, GEO)
    assert d == 0
    i = 11
    g = oracle.features(tr[:, 0], i, W, GEO)
    o = oracle.mlp(g, W)
    assert np.array_equal(H[100 * i:100 * (i + 1)], o)
    H2 = H.copy()
    H2[100 * i:100 * (i + 1)] = 0
    assert not np.any(H2)
    assert np.all(o > 0)                      # softplus outputs are positive


def test_mass_and_empty_bins():
    tr = _event(3)
    H, d = oracle.histogram(tr, W, GEO)
    total = 0.0
    filled = set()
    for t in range(tr.shape[1]):
        i = oracle.bin_index(tr[0, t], GEO)
        if i < 0:
            continue
        filled.add(i)
        total += oracle.mlp(oracle.features(tr[:, t], i, W, GEO), W).sum()
    assert H.sum() == pytest.approx(total, rel=1e-13)
    for i in range(40):
        seg = H[100 * i:100 * (i + 1)]
        assert (np.all(seg > 0) if i in filled else not np.any(seg))


def test_dropped_tracks():
    tr = _event(0)[:, :6].copy()
    tr[0, 0] = np.float32(-100.5)              # below the window
    tr[0, 1] = np.float32(300.0)               # upper edge is outside
    tr[4, 2] = np.float32("nan")               # a non-finite feature
    tr[7, 3] = np.float32("inf")
    H, d = oracle.histogram(tr, W, GEO)
    assert d == 4
    Hk, dk = oracle.histogram(tr[:, 4:], W, GEO)
    assert dk == 0 and np.array_equal(H, Hk)


def test_zero_tracks():
    H, d = oracle.histogram(np.zeros((9, 0), np.float32), W, GEO)
    assert d == 0 and not np.any(H)
