"""The seeded input generator: determinism, layout and the workload statistics
the paper states (5.6 primary vertices per event on average, Section 1)."""

import numpy as np
import pytest

from synth import make_events, make_weights, weights_to_blob, NetShape
from synth.events import pack_events


def test_events_deterministic_and_prefix_stable():
    a = make_events(12, seed=0)
    b = make_events(12, seed=0)
    assert np.array_equal(a.feat, b.feat) and np.array_equal(a.offsets, b.offsets)
    c = make_events(5, seed=0)
    assert np.array_equal(c.feat, a.feat[:, :c.offsets[-1]])
    d = make_events(5, seed=1)
    assert not np.array_equal(c.feat[:, :10], d.feat[:, :10])


def test_events_layout():
    ev = make_events(20, seed=3)
    assert ev.feat.dtype == np.float32 and ev.feat.flags.c_contiguous
    assert ev.feat.shape == (9, ev.offsets[-1])
    assert ev.offsets.dtype == np.int32 and ev.offsets[0] == 0
    assert np.all(np.diff(ev.offsets) >= 0)
    sub = ev.subset([4, 2])
    assert np.array_equal(sub.tracks_of(0), ev.tracks_of(4))
    assert np.array_equal(sub.tracks_of(1), ev.tracks_of(2))


def test_event_statistics():
    ev = make_events(2000, seed=0)
    T = np.diff(ev.offsets)
    assert abs(T.mean() - 180.0) < 1.5
    npv = np.array([len(z) for z in ev.pv_z])
    assert npv.min() >= 1
    # zero-truncated Poisson(5.6) has mean 5.6 / (1 - exp(-5.6))
    assert abs(npv.mean() - 5.6 / (1 - np.exp(-5.6))) < 0.15
    allz = np.concatenate(ev.pv_z)
    assert allz.min() >= -100 and allz.max() <= 300
    assert abs(allz.std() - 45.0) < 2.0
    c = ev.feat[3:6].ravel().astype(np.float64)
    assert abs(np.log(c).mean() + 3.0) < 0.01 and abs(np.log(c).std() - 0.5) < 0.01
    s = ev.feat[6:9].ravel()
    assert abs(s.std() - 0.2) < 0.002


def test_heavy_tailed_mix():
    ev = make_events(3000, seed=0, mix="lognormal")
    T = np.diff(ev.offsets)
    assert T.min() >= 5 and T.max() <= 1500
    assert abs(np.median(T) - 180) < 12
    assert (T == 1500).mean() > 0.005


def test_weights_deterministic_and_he_scaled():
    w = make_weights(0)
    w2 = make_weights(0)
    for n, shp, fan_in in w.shape.tensor_list():
        assert w[n].shape == shp and w[n].dtype == np.float32
        assert np.array_equal(w[n], w2[n])
        if n.endswith(".b"):
            assert np.all(np.abs(w[n]) <= 1 / np.sqrt(fan_in) + 1e-7)
    big = w["enc3.c2.w"]
    assert abs(big.std() - np.sqrt(2 / (256 * 5))) < 0.002
    wz = make_weights(0, zero_bias=True)
    assert np.array_equal(wz["enc0.c1.w"], w["enc0.c1.w"])
    assert not np.any(wz["dec0.c2.b"])


def test_parameter_count():
    w = make_weights(0)
    n_unet = sum(w[n].size for n, _, _ in w.shape.tensor_list() if not n.startswith("mlp"))
    assert 1_000_000 < n_unet < 1_100_000


def test_blob_layout():
    w = make_weights(0)
    blob = weights_to_blob(w)
    assert blob[:4] == b"PVFW"
    names = [n for n, _, _ in w.shape.tensor_list()]
    n_floats = sum(w[n].size for n in names)
    header = 4 + 4 + 7 * 4 + 2 * 4 + 18 * 4 + 4 + 4 * len(names)
    assert len(blob) == header + 4 * n_floats
    tail = np.frombuffer(blob[-4 * w["head.b"].size:], dtype="<f4")
    assert np.array_equal(tail, w["head.b"])


def test_pack_events_handles_empty():
    ev = pack_events([np.zeros((9, 0), np.float32), np.ones((9, 3), np.float32)])
    assert list(ev.offsets) == [0, 0, 3]
