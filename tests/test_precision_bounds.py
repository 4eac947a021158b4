"""Derivation of the reduced-precision tolerances (tests/parity.py) from a CPU
emulation of the BF16, FP16 and FP8 arithmetic (tests/emulate.py) against the
FP64 oracle.

The paper's Section 5 proposes FP16 on the matrix units without stating an
accuracy target for the network output, so each bound is set from what the
rounding itself does to this network: the emulation rounds exactly where the
kernels round (weights, stored activations, track-network layer inputs;
FP32 accumulation; head and sigmoid in FP32) and the bound must sit above the
emulated error with a stated margin, and not far above it:

    MARGIN_LO * emulated max|dp|  <=  bound  <=  MARGIN_HI * emulated max|dp|

Vertex agreement (|dz| <= 0.05 mm, one-to-one) must be at least the stated
floor, which sits below the emulated match rate; unmatched GPU vertices at
most the stated ceiling, above the emulated extra rate.  The GPU tests then
hold the kernels to these bounds.
"""

import numpy as np
import pytest

import oracle
from synth import make_events, make_weights, NetShape
from tests import emulate, parity

pytestmark = pytest.mark.slow

MARGIN_LO = 1.15
MARGIN_HI = 4.0
WIDE = NetShape(base_channels=64)


def vertex_rates(p, refs, geo=oracle.Geometry()):
    m = tot = extra = 0
    for e, ref in enumerate(refs):
        pk = oracle.peaks(p[e], geo)
        k = parity.match_vertices(pk["z"], ref["z"])
        m += k
        extra += len(pk["z"]) - k
        tot += len(ref["z"])
    return m / tot, extra / tot


def max_dp(p, refs):
    return max(float(np.max(np.abs(p[e] - r["p"]))) for e, r in enumerate(refs))


def events_of(batch):
    return [batch.tracks_of(e) for e in range(batch.n_events)]


@pytest.fixture(scope="module")
def seed0():
    w = make_weights(0)
    b = make_events(16, seed=0)
    cal = emulate.calibrate(events_of(make_events(64, seed=5)), w)
    return w, events_of(b), oracle.run_batch(b, w), cal


def test_emulation_in_fp32_is_the_oracle(seed0):
    """Without rounding, the emulation is the same network as the oracle
    (float32 arithmetic): p within 1e-5 relative."""
    w, ev, refs, _ = seed0
    p = emulate.forward(ev, w, "fp32")
    assert max(parity.max_rel(p[e], refs[e]["p"]) for e in range(len(ev))) <= 1e-5


def test_rounding_is_what_the_emulation_says():
    """The rounding helpers: BF16 and FP16 round to nearest even, e4m3 too,
    saturating at 448; 17 lies halfway between the e4m3 values 16 and 18."""
    import torch
    x = torch.tensor([17.0, 19.0, 449.0, -1000.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8])
    assert emulate._round(x, "fp8_e4m3").tolist() == [16.0, 20.0, 448.0, -448.0, 1.0, 1.0]
    assert emulate._round(x[4:], "bf16").tolist() == [1.0, 1.0 + 2 ** -6]
    assert emulate._round(torch.tensor([1.0 + 2 ** -11]), "fp16").tolist() == [1.0]


@pytest.mark.parametrize("dt", ["bf16", "fp16", "fp8_e4m3"])
def test_bounds_of_the_1000_event_network(seed0, dt):
    """The 4000-bin, 32..256-channel network on the 16 seed-0 events."""
    w, ev, refs, cal = seed0
    p = emulate.forward(ev, w, dt, cal if dt == "fp8_e4m3" else None)
    dp = max_dp(p, refs)
    match, extra = vertex_rates(p, refs)
    print(f"{dt}: emulated max|dp| {dp:.4e} (bound {parity.P_ABS[dt]}), matched {match:.4f} "
          f"(floor {parity.MATCH_MIN[dt]}), extra {extra:.4f} (ceiling {parity.EXTRA_MAX[dt]})")
    assert MARGIN_LO * dp <= parity.P_ABS[dt] <= MARGIN_HI * dp
    assert parity.MATCH_MIN[dt] < match
    assert extra < parity.EXTRA_MAX[dt]


@pytest.mark.parametrize("dt", ["bf16", "fp16", "fp8_e4m3"])
def test_bounds_of_the_64_channel_network(dt):
    """The paper's deployed 64-channel width on 6 seed-1 events (FP8 scales
    from 32 events of seed 5)."""
    w = make_weights(0, shape=WIDE)
    b = make_events(6, seed=1)
    refs = oracle.run_batch(b, w)
    cal = emulate.calibrate(events_of(make_events(32, seed=5)), w) if dt == "fp8_e4m3" else None
    p = emulate.forward(events_of(b), w, dt, cal)
    dp = max_dp(p, refs)
    match, _ = vertex_rates(p, refs)
    print(f"{dt} (64 channels): emulated max|dp| {dp:.4e} (bound {parity.P_ABS_WIDE[dt]}), "
          f"matched {match:.4f} (floor {parity.MATCH_MIN_WIDE[dt]})")
    assert MARGIN_LO * dp <= parity.P_ABS_WIDE[dt] <= MARGIN_HI * dp
    assert parity.MATCH_MIN_WIDE[dt] < match


def heavy_events():
    """The heavy-tailed 4096-event batch (log-normal track counts): every
    event of at least 1000 tracks (168 of them, 68 clipped at 1500), where
    the network's logits are largest, and the sampled events of the GPU test
    (first, last, largest, smallest, four random)."""
    b = make_events(4096, seed=0, mix="lognormal")
    T = np.diff(b.offsets)
    rng = np.random.default_rng(4096)
    sample = set([0, 4095, int(np.argmax(T)), int(np.argmin(T))] + rng.choice(4096, 4, replace=False).tolist())
    idx = sorted(sample | set(np.nonzero(T >= 1000)[0].tolist()))
    return b.subset(idx)


def test_bounds_of_the_heavy_tailed_batch():
    """BF16 on heavy-tailed events: events of 1000-1500 tracks drive the
    logits beyond 100, so the absolute rounding error of the deep layers
    moves p by more than on the Poisson(180) events."""
    w = make_weights(0)
    b = heavy_events()
    refs = oracle.run_batch(b, w)
    p = emulate.forward(events_of(b), w, "bf16")
    dp = max_dp(p, refs)
    match, extra = vertex_rates(p, refs)
    print(f"bf16 heavy-tailed: emulated max|dp| {dp:.4e} (bound {parity.P_ABS_HEAVY['bf16']}), "
          f"matched {match:.4f} (floor {parity.MATCH_MIN_HEAVY['bf16']}), extra {extra:.4f}")
    assert MARGIN_LO * dp <= parity.P_ABS_HEAVY["bf16"] <= MARGIN_HI * dp
    assert parity.MATCH_MIN_HEAVY["bf16"] < match
    assert extra < parity.EXTRA_MAX["bf16"]
