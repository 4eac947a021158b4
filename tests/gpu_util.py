"""Shared helpers of the GPU tests: engines, uploads, oracle references."""

import functools

import numpy as np

import oracle
from synth import make_events, make_weights, weights_to_blob


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


@functools.lru_cache(maxsize=None)
def weights(seed=0, shape=None):
    return make_weights(seed) if shape is None else make_weights(seed, shape=shape)


@functools.lru_cache(maxsize=None)
def blob(seed=0, shape=None):
    return weights_to_blob(weights(seed, shape))


def make_engine(max_events, fp8_amax=None, shape=None, **spec):
    """Engine for `max_events`; `shape` (a synth NetShape) selects the
    network (its levels and width go into the spec too)."""
    import paper_2602_19959_amd as pv
    if shape is not None:
        spec.setdefault("n_levels", shape.n_levels)
        spec.setdefault("base_channels", shape.base_channels)
    s = pv.default_spec(max_events=max_events, **spec)
    if "max_tracks_total" not in spec:
        s.max_tracks_total = max_events * 1500
    return pv.Engine(blob(0, shape), s, fp8_amax=fp8_amax)


@functools.lru_cache(maxsize=None)
def fp8_calibration(n_events=64, seed=5, shape=None):
    """Calibration table of an FP32 engine over `n_events` events of `seed`
    (events the FP8 tests never score)."""
    import paper_2602_19959_amd as pv
    batch = make_events(n_events, seed=seed)
    eng = make_engine(n_events, shape=shape)
    feat, off = pv.upload_events(batch)
    amax = eng.calibrate(feat, off)
    eng.close()
    return amax


def engine_for(max_events, dtype, **spec):
    """Engine of any compute dtype; FP8 gets the standard calibration table."""
    amax = fp8_calibration() if dtype == "fp8_e4m3" else None
    return make_engine(max_events, fp8_amax=amax, compute_dtype=dtype, **spec)


def run(engine, batch, with_prob=True):
    """Upload `batch`, execute, wait, return host numpy outputs."""
    import paper_2602_19959_amd as pv
    feat, off = pv.upload_events(batch)
    out = engine.alloc_outputs(batch.n_events, with_prob=with_prob)
    engine.execute(feat, off, out)
    engine.synchronize()
    return out.to_host()


def geometry(engine):
    s = engine.spec
    return oracle.Geometry(z_min=s.z_min_mm, bin_width=s.bin_width_mm,
                           n_intervals=s.n_bins // s.bins_per_interval,
                           bins_per_interval=s.bins_per_interval, p_min=s.peak_min,
                           s_min=s.integral_min, half_window=s.half_window,
                           max_peaks=s.max_peaks_per_event, boundary_mm=s.boundary_mm,
                           layout=("event", "interval")[s.unet_layout])


def event_vertices(host, e):
    """(bins, z, height, window sum) of event e's vertices."""
    n = int(host["n_vertices"][e])
    return host["bin"][e, :n], host["z"][e, :n], host["peak_prob"][e, :n], host["integral"][e, :n]
