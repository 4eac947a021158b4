"""Pins of the oracle's UNet (Section 2: the encoder lowers the resolution and
raises the channel depth, the decoder upsamples back to a per-bin output).

* An event with no track has an all-zero histogram.  Then every encoder map
  is constant along z away from the ends, each stride-2 upsampling doubles the
  period, and the output is 8-periodic in the interior.  Its values follow a
  "phase recursion" on per-channel vectors of period P, written here from the
  definitions with modular indexing, independent of the oracle's sliding
  windows.
* With every bias zero, a zero input stays exactly zero, so p = 1/2.
* A change to one input bin moves only outputs within the network's
  receptive field.
"""

import numpy as np
import pytest

import oracle
from synth import make_weights, make_events
from tests import torch_ref

W = make_weights(0)
L = 4000


def lrelu(x, s):
    return np.where(x >= 0, x, s * x)


def periodic_conv(x, Wt, b):
    """x [Cin][P] periodic; 5-tap same correlation in the periodic interior."""
    Cout, Cin, k = Wt.shape
    P = x.shape[1]
    r = (k - 1) // 2
    y = np.zeros((Cout, P))
    for phi in range(P):
        for j in range(k):
            y[:, phi] += Wt[:, :, j].astype(np.float64) @ x[:, (phi + j - r) % P]
    return y + b.astype(np.float64)[:, None]


def periodic_up(x, WT, b):
    """stride-2 2-tap transposed conv of a P-periodic map: 2P-periodic."""
    Cin, Cout, _ = WT.shape
    P = x.shape[1]
    y = np.zeros((Cout, 2 * P))
    for phi in range(2 * P):
        y[:, phi] = WT[:, :, phi % 2].astype(np.float64).T @ x[:, phi // 2]
    return y + b.astype(np.float64)[:, None]


def phase_recursion(w):
    s = w.shape
    x = np.zeros((1, 1))
    skips = []
    for lv in range(s.n_levels):
        for j in (1, 2):
            x = lrelu(periodic_conv(x, w[f"enc{lv}.c{j}.w"], w[f"enc{lv}.c{j}.b"]), w.leaky)
        skips.append(x)            # period 1: max-pool of a constant is the constant
    for lv in range(s.n_levels - 2, -1, -1):
        u = periodic_up(x, w[f"up{lv}.w"], w[f"up{lv}.b"])
        P = u.shape[1]
        sk = np.tile(skips[lv], (1, P // skips[lv].shape[1]))
        x = np.concatenate([sk, u], 0)
        for j in (1, 2):
            x = lrelu(periodic_conv(x, w[f"dec{lv}.c{j}.w"], w[f"dec{lv}.c{j}.b"]), w.leaky)
    return w["head.w"].astype(np.float64)[0] @ x + float(w["head.b"][0])


@pytest.fixture(scope="module")
def zero_event_logit():
    return oracle.unet(np.zeros(L), W)


def test_zero_track_interior_is_8_periodic_and_matches_phase_recursion(zero_event_logit):
    logit = zero_event_logit
    per = phase_recursion(W)
    assert per.shape == (8,)
    margin = 128
    t = np.arange(margin, L - margin)
    np.testing.assert_allclose(logit[t], per[t % 8], rtol=1e-12, atol=1e-13)
    # the ends differ from the periodic pattern (zero padding reaches them)
    assert np.abs(logit[:4] - per[np.arange(4) % 8]).max() > 1e-6


def test_zero_track_event_end_to_end(zero_event_logit):
    r = oracle.run_event(np.zeros((9, 0), np.float32), W)
    assert not np.any(r["H"])
    np.testing.assert_array_equal(r["logit"], zero_event_logit)


def test_zero_bias_zero_input_gives_one_half():
    wz = make_weights(0, zero_bias=True)
    r = oracle.run_event(np.zeros((9, 0), np.float32), wz)
    assert np.all(r["logit"] == 0.0) and np.all(r["p"] == 0.5)


def _influence(t0, shape):
    """Interval of outputs an input bin t0 can reach: a 5-tap conv widens an
    interval by 2 each side, pooling maps [a, b] to [a//2, b//2], the stride-2
    upsampling maps [a, b] to [2a, 2b+1], a concatenation takes the union."""
    x, skips = (t0, t0), []
    for lv in range(shape.n_levels):
        for _ in (1, 2):
            x = (x[0] - 2, x[1] + 2)
        skips.append(x)
        if lv < shape.n_levels - 1:
            x = (x[0] // 2, x[1] // 2)
    for lv in range(shape.n_levels - 2, -1, -1):
        x = (min(skips[lv][0], 2 * x[0]), max(skips[lv][1], 2 * x[1] + 1))
        for _ in (1, 2):
            x = (x[0] - 2, x[1] + 2)
    return x


def test_receptive_field():
    x = np.random.default_rng(7).uniform(0, 2, L)
    base = oracle.unet(x, W)
    for t0 in (2000, 2007):
        x2 = x.copy()
        x2[t0] += 1.0
        moved = np.nonzero(oracle.unet(x2, W) != base)[0]
        lo, hi = _influence(t0, W.shape)
        assert (lo, hi) == ((1908, 2091) if t0 == 2000 else (1916, 2099))
        assert moved.min() == lo and moved.max() == hi


def test_taps_shapes_and_consistency():
    x = np.random.default_rng(8).uniform(0, 2, L)
    taps = oracle.unet_taps(x, W)
    assert taps["enc0.c1"].shape == (32, 4000)
    assert taps["enc3.c2"].shape == (256, 500)
    assert taps["up2"].shape == (128, 1000)
    np.testing.assert_array_equal(taps["logit"], oracle.unet(x, W))
    np.testing.assert_array_equal(taps["pool0"], oracle.maxpool2(taps["enc0.c2"]))


def test_unet_vs_torch_restatement():
    x = np.random.default_rng(9).uniform(0, 3, L)
    np.testing.assert_allclose(oracle.unet(x, W), torch_ref.unet(x, W).numpy(), rtol=1e-11, atol=1e-12)
