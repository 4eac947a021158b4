"""Pins of the oracle's building blocks against the mathematics and against
library routines (not against the oracle itself).

Section 2 of the paper defines the pipeline: per-track FC layers, a UNet of
1D convolutions with pooling down and upsampling back, then peak finding.
The readings of the silent details (same padding, cross-correlation, 2-tap
stride-2 upsampling, LeakyReLU, softplus outputs, interval-local z feature)
are stated in the oracle's header.
"""

import json
import math
import os
import struct

import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
from synth import make_weights, NetShape, Weights

GOLD = os.path.join(os.path.dirname(__file__), "golden")
rng = np.random.default_rng(1234)


def brute_conv1d(x, W, b):
    """Direct definition of same-padded cross-correlation, written as nested
    Python loops (tiny inputs only)."""
    Cout, Cin, k = W.shape
    L = x.shape[1]
    r = (k - 1) // 2
    y = np.zeros((Cout, L))
    for o in range(Cout):
        for t in range(L):
            s = float(b[o])
            for c in range(Cin):
                for j in range(k):
                    u = t + j - r
                    if 0 <= u < L:
                        s += float(W[o, c, j]) * float(x[c, u])
            y[o, t] = s
    return y


@pytest.mark.parametrize("Cin,Cout,L,k", [(1, 1, 8, 5), (2, 3, 9, 5), (3, 2, 16, 5),
                                          (1, 4, 5, 5), (2, 2, 3, 5), (3, 1, 7, 3), (2, 2, 6, 1)])
def test_conv1d_brute_force(Cin, Cout, L, k):
    x = rng.normal(size=(Cin, L))
    W = rng.normal(size=(Cout, Cin, k)).astype(np.float32)
    b = rng.normal(size=Cout).astype(np.float32)
    np.testing.assert_allclose(oracle.conv1d(x, W, b), brute_conv1d(x, W, b), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("Cin,Cout,L", [(1, 32, 40), (32, 32, 37), (64, 16, 50), (5, 7, 2)])
def test_conv1d_vs_torch(Cin, Cout, L):
    x = rng.normal(size=(Cin, L))
    W = rng.normal(size=(Cout, Cin, 5)).astype(np.float32)
    b = rng.normal(size=Cout).astype(np.float32)
    ref = F.conv1d(torch.tensor(x)[None], torch.tensor(W, dtype=torch.float64),
                   torch.tensor(b, dtype=torch.float64), padding=2)[0].numpy()
    np.testing.assert_allclose(oracle.conv1d(x, W, b), ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("Cin,Cout,L", [(2, 1, 4), (8, 4, 11), (64, 32, 25)])
def test_convT2_vs_torch(Cin, Cout, L):
    x = rng.normal(size=(Cin, L))
    W = rng.normal(size=(Cin, Cout, 2)).astype(np.float32)
    b = rng.normal(size=Cout).astype(np.float32)
    ref = F.conv_transpose1d(torch.tensor(x)[None], torch.tensor(W, dtype=torch.float64),
                             torch.tensor(b, dtype=torch.float64), stride=2)[0].numpy()
    np.testing.assert_allclose(oracle.convT2(x, W, b), ref, rtol=1e-12, atol=1e-12)


def test_convT2_equals_interleave_then_correlate():
    """Identity: a stride-2, 2-tap transposed conv equals zero-interleaving the
    input and correlating with the kernel taps reversed (k=2, no padding on
    the left, one zero on the right)."""
    Cin, Cout, L = 3, 2, 6
    x = rng.normal(size=(Cin, L))
    W = rng.normal(size=(Cin, Cout, 2)).astype(np.float32)
    b = rng.normal(size=Cout).astype(np.float32)
    z = np.zeros((Cin, 2 * L + 1))
    z[:, 1::2] = x                    # x[t] sits at 2t+1; a zero at index 0
    y = np.zeros((Cout, 2 * L))
    for o in range(Cout):
        for s in range(2 * L):
            acc = float(b[o])
            for c in range(Cin):
                # y[s] = sum_j W[c][o][j] * x[(s-j)/2] over j with s-j even
                acc += float(W[c, o, 0]) * z[c, s + 1] + float(W[c, o, 1]) * z[c, s]
            y[o, s] = acc
    np.testing.assert_allclose(oracle.convT2(x, W, b), y, rtol=1e-13, atol=1e-13)


def test_sigmoid_closed_forms_and_library():
    """The head's logistic function (Section 2: the UNet ends in a per-bin
    probability): sigma(ln 3) = 3/4 and sigma(-ln 3) = 1/4 (exp(-ln 3) = 1/3),
    sigma(0) = 1/2, increasing, and equal to torch.sigmoid in float64."""
    ln3 = math.log(3.0)
    assert abs(oracle.sigmoid(ln3) - 0.75) <= 2e-16
    assert abs(oracle.sigmoid(-ln3) - 0.25) <= 2e-16
    assert oracle.sigmoid(0.0) == 0.5
    x = np.linspace(-30.0, 30.0, 601)
    s = oracle.sigmoid(x)
    assert np.all(np.diff(s) > 0)
    ref = torch.sigmoid(torch.from_numpy(x)).numpy()
    np.testing.assert_allclose(s, ref, rtol=1e-15, atol=0)


def test_maxpool2_vs_torch():
    x = rng.normal(size=(5, 20))
    ref = F.max_pool1d(torch.tensor(x)[None], 2)[0].numpy()
    assert np.array_equal(oracle.maxpool2(x), ref)


def _tiny_weights(tensors, shape):
    return Weights(shape, {k: np.asarray(v, np.float32) for k, v in tensors.items()})


def test_mlp_closed_forms():
    shape = NetShape(n_feat=1, hidden=1, n_hidden=1, n_out=1)
    # identity weights: out = softplus(LReLU(g))
    w = _tiny_weights({"mlp0.w": [[1.0]], "mlp0.b": [0.0], "mlp1.w": [[1.0]], "mlp1.b": [0.0]}, shape)
    w.leaky = 0.01
    assert oracle.mlp([0.0], w)[0] == pytest.approx(math.log(2.0), rel=1e-15)
    assert oracle.mlp([-1.0], w)[0] == pytest.approx(math.log1p(math.exp(-0.01)), rel=1e-15)
    assert oracle.mlp([3.0], w)[0] == pytest.approx(math.log1p(math.exp(3.0)), rel=1e-15)
    # softplus must not overflow or lose the linear tail
    assert oracle.mlp([800.0], w)[0] == pytest.approx(800.0, rel=1e-15)
    assert oracle.mlp([-800.0], w)[0] == pytest.approx(math.log1p(math.exp(-8.0)), rel=1e-15)


def test_mlp_vs_torch():
    w = make_weights(0)
    s = w.shape
    for _ in range(20):
        g = rng.normal(size=s.n_feat) * 2
        h = torch.tensor(g)
        for l in range(s.n_hidden):
            h = F.leaky_relu(F.linear(h, torch.tensor(w[f"mlp{l}.w"], dtype=torch.float64),
                                      torch.tensor(w[f"mlp{l}.b"], dtype=torch.float64)), w.leaky)
        o = F.softplus(F.linear(h, torch.tensor(w[f"mlp{s.n_hidden}.w"], dtype=torch.float64),
                                torch.tensor(w[f"mlp{s.n_hidden}.b"], dtype=torch.float64)))
        np.testing.assert_allclose(oracle.mlp(g, w), o.numpy(), rtol=1e-13)


def _golden_z(c):
    if "z_bits" in c:
        return struct.unpack("<f", struct.pack("<I", int(c["z_bits"], 16)))[0]
    return float(np.float32(float(c["z"])))


def test_bin_edges_golden():
    g = json.load(open(os.path.join(GOLD, "bin_edges.json")))
    geo = oracle.Geometry()
    for c in g["cases"]:
        assert oracle.bin_index(_golden_z(c), geo) == c["interval"], c


def test_features_closed_form():
    w = make_weights(0)
    geo = oracle.Geometry()
    tr = np.array([-95.0, 0.064, -0.128, 0.0864, 0.0564, 0.0264, 0.2, -0.4, 0.0], np.float32)
    g = oracle.features(tr, 0, w, geo)
    assert g[0] == 0.0                                   # centre of interval 0
    assert g[1] == pytest.approx(float(np.float32(0.064)) * w.scale[1], rel=1e-15)
    assert g[3] == pytest.approx((float(np.float32(0.0864)) - w.shift[3]) * w.scale[3], rel=1e-12)
    assert oracle.features(np.r_[np.float32(-100.0), tr[1:]], 0, w, geo)[0] == -1.0
    g = oracle.features(np.r_[np.float32(2.5), tr[1:]], 10, w, geo)
    assert g[0] == -0.5                                   # a quarter into interval 10
