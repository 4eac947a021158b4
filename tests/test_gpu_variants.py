"""The paper's Section 3/5 variants on the GPU against the FP64 oracle, through
the C ABI: the 64-channel UNet width (the paper's deployed network), boundary
tracks that feed two intervals, and the interval-batched UNet layout.  Bars as
for the main path (tests/parity.py): FP32 p within 1e-4 relative and the same
peaks on every robust decision; reduced precision within its stated bounds."""

import dataclasses

import numpy as np
import pytest

import oracle
from synth import make_events, NetShape
from synth.events import pack_events
from tests import parity
from tests.gpu_util import (torch_cuda, make_engine, run, geometry, event_vertices, weights,
                            fp8_calibration)

pytestmark = pytest.mark.gpu

WIDE = NetShape(base_channels=64)
L3 = NetShape(n_levels=3)


def say(*a):
    print("[gpu-variants]", *a, flush=True)


def check_fp32(eng, batch, out, w):
    geo = geometry(eng)
    refs = oracle.run_batch(batch, w, geo)
    amb_total = 0
    for e in range(batch.n_events):
        err = parity.max_rel(out["prob"][e], refs[e]["p"])
        assert err <= parity.P_REL, (e, err)
        bins, z, h, S = event_vertices(out, e)
        amb, _ = parity.compare_peaks(bins, z, h, S, refs[e], geo)
        amb_total += amb
    parity.exact_peaks_all(out, geo)
    return refs, amb_total


# ---------------------------------------------------------------- width 64

def test_wide_unet_fp32():
    torch_cuda()
    batch = make_events(6, seed=1)
    say("64-channel UNet, FP32, 6 events")
    eng = make_engine(6, shape=WIDE)
    out = run(eng, batch)
    refs, amb = check_fp32(eng, batch, out, weights(0, WIDE))
    say("ambiguous decisions excluded:", amb)
    # a deep layer of event 0, normwise
    w = weights(0, WIDE)
    taps = oracle.unet_taps(w.s_in * refs[0]["H"], w)
    run(eng, batch.subset([0]))
    for name in ("enc3.c2", "dec0.c1"):
        got = eng.debug_tensor(name, 1).cpu().numpy().reshape(taps[name].shape)
        assert parity.tap_err(got, taps[name]) <= parity.TAP_NORM, name
    assert np.array_equal(run(eng, batch)["prob"], out["prob"])
    eng.close()


@pytest.mark.parametrize("dt", ["bf16", "fp8_e4m3"])
def test_wide_unet_low_precision(dt):
    torch_cuda()
    batch = make_events(6, seed=1)
    w = weights(0, WIDE)
    refs = oracle.run_batch(batch, w)
    amax = fp8_calibration(32, 5, WIDE) if dt == "fp8_e4m3" else None
    say("64-channel UNet", dt)
    eng = make_engine(6, shape=WIDE, compute_dtype=dt, fp8_amax=amax)
    out = run(eng, batch)
    dp = max(float(np.max(np.abs(out["prob"][e] - refs[e]["p"]))) for e in range(6))
    matched = total = 0
    for e in range(6):
        n = int(out["n_vertices"][e])
        matched += parity.match_vertices(out["z"][e, :n], refs[e]["z"])
        total += len(refs[e]["z"])
    say(dt, "max |dp| %.3e, vertices matched %d/%d" % (dp, matched, total))
    assert dp <= parity.P_ABS_WIDE[dt]
    assert matched >= parity.MATCH_MIN_WIDE[dt] * total
    parity.exact_peaks_all(out, geometry(eng))
    eng.close()


# ---------------------------------------------------------------- boundary tracks

@pytest.mark.parametrize("b", [1.0, 5.0])
def test_boundary_tracks_fp32(b):
    torch_cuda()
    batch = make_events(8, seed=2)
    say(f"boundary {b} mm, FP32, 8 events")
    eng = make_engine(8, boundary_mm=b)
    out = run(eng, batch)
    refs, amb = check_fp32(eng, batch, out, weights())
    hist = eng.debug_tensor("hist", 8).cpu().numpy().reshape(8, -1)
    s_in = weights().s_in
    for e in range(8):
        ref = s_in * refs[e]["H"]
        nz = ref != 0
        assert np.all(hist[e][~nz] == 0)
        assert parity.max_rel(hist[e][nz], ref[nz]) <= parity.P_REL
    # the second-interval terms are really there: the one-interval histogram differs
    plain = oracle.histogram(batch.tracks_of(0), weights())[0] * s_in
    assert np.max(np.abs(hist[0] - plain)) > 1e-2 * np.max(np.abs(plain))
    say("ambiguous decisions excluded:", amb)
    # deterministic and batch-invariant with the staging pass
    assert np.array_equal(run(eng, batch)["prob"], out["prob"])
    alone = run(eng, batch.subset([3]))
    assert np.array_equal(alone["prob"][0], out["prob"][3])
    eng.close()


def test_boundary_tracks_bf16():
    """Boundary tracks through the matrix-core network and the register
    histogram: the BF16 histogram within BF16 rounding of the oracle's
    (normwise), the neighbour terms present, p within the BF16 bound, and the
    result deterministic and batch-invariant with the staging pass."""
    torch_cuda()
    b = 5.0
    batch = make_events(8, seed=2)
    say(f"boundary {b} mm, BF16, 8 events")
    eng = make_engine(8, boundary_mm=b, compute_dtype="bf16")
    assert eng.launch_kernels()[0].startswith("track_stage_mma<")
    out = run(eng, batch)
    w = weights()
    refs = oracle.run_batch(batch, w, geometry(eng))
    hist = eng.debug_tensor("hist", 8).cpu().numpy().reshape(8, -1)
    for e in range(8):
        err = parity.tap_err(hist[e], w.s_in * refs[e]["H"])
        assert err <= 3e-2, (e, err)
        assert float(np.max(np.abs(out["prob"][e] - refs[e]["p"]))) <= parity.P_ABS["bf16"], e
    plain = oracle.histogram(batch.tracks_of(0), w)[0] * w.s_in
    assert np.max(np.abs(hist[0] - plain)) > 1e-2 * np.max(np.abs(plain))
    assert np.array_equal(run(eng, batch)["prob"], out["prob"])
    alone = run(eng, batch.subset([3]))
    assert np.array_equal(alone["prob"][0], out["prob"][3])
    eng.close()


def test_boundary_decisions_at_the_edges():
    """Tracks placed at, just inside and just outside the boundary distance of
    shared and outer edges: the intervals each event touches (non-zero bins)
    are exactly the oracle's."""
    torch_cuda()
    b = 1.0
    zs = [-50.0 + 1.0, -50.0 + 1.0 - 2 ** -18, -50.0 + 1.0 + 2 ** -18, -50.0, -50.0 - 2 ** -18,
          -41.0, -41.0 - 2 ** -18, -41.0 + 2 ** -18, -100.0, -99.5, 299.5, 299.0 - 2 ** -16, 0.0]
    rng = np.random.default_rng(4)
    lists = []
    for z in zs:
        t = np.zeros((9, 1), np.float32)
        t[0, 0] = z
        t[1:3, 0] = rng.normal(0, 0.05, 2)
        t[3:6, 0] = rng.normal(0, 0.3, 3)
        t[6:9, 0] = np.abs(rng.normal(0.05, 0.02, 3))
        lists.append(t)
    batch = pack_events(lists)
    eng = make_engine(len(zs), boundary_mm=b)
    run(eng, batch)
    hist = eng.debug_tensor("hist", len(zs)).cpu().numpy().reshape(len(zs), 40, 100)
    geo = geometry(eng)
    for k, t in enumerate(lists):
        ref = oracle.histogram(t, weights(), geo)[0].reshape(40, 100)
        got_on = [i for i in range(40) if np.any(hist[k, i] != 0)]
        ref_on = [i for i in range(40) if np.any(ref[i] != 0)]
        assert got_on == ref_on, (zs[k], got_on, ref_on)
    eng.close()


# ---------------------------------------------------------------- interval layout

@pytest.mark.parametrize("b", [0.0, 2.5])
def test_interval_layout_fp32(b):
    torch_cuda()
    batch = make_events(6, seed=3)
    say(f"interval layout, 3 levels, boundary {b} mm, FP32")
    eng = make_engine(6, shape=L3, unet_layout="interval", boundary_mm=b)
    out = run(eng, batch)
    refs, amb = check_fp32(eng, batch, out, weights(0, L3))
    say("ambiguous decisions excluded:", amb)
    # the per-interval UNet differs from the event-wide one
    ev = oracle.run_event(batch.tracks_of(0), weights(0, L3),
                          dataclasses.replace(geometry(eng), layout="event"))
    assert np.max(np.abs(out["prob"][0] - ev["p"])) > 1e-3
    alone = run(eng, batch.subset([4]))
    assert np.array_equal(alone["prob"][0], out["prob"][4])
    eng.close()


def test_interval_layout_bf16():
    torch_cuda()
    batch = make_events(6, seed=3)
    eng = make_engine(6, shape=L3, unet_layout="interval", compute_dtype="bf16")
    out = run(eng, batch)
    refs = oracle.run_batch(batch, weights(0, L3), geometry(eng))
    dp = max(float(np.max(np.abs(out["prob"][e] - refs[e]["p"]))) for e in range(6))
    say("interval layout bf16 max |dp| %.3e" % dp)
    assert dp <= parity.P_ABS["bf16"]
    parity.exact_peaks_all(out, geometry(eng))
    eng.close()
