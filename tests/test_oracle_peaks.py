"""Pins of the oracle's peak finder (Section 2: local-maximum detection with
thresholds) against hand-derived cases and against scipy's find_peaks."""

import json
import os

import numpy as np
import pytest
from scipy.signal import find_peaks

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _cases():
    return json.load(open(os.path.join(GOLD, "peaks_hand.json")))["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_hand_cases(case):
    g = case["geo"]
    geo = oracle.Geometry(z_min=g["z_min"], bin_width=g["bw"], p_min=g["p_min"], s_min=g["s_min"],
                          half_window=g["hw"], n_intervals=1, bins_per_interval=g["L"])
    p = np.zeros(g["L"])
    for k, v in case["p"].items():
        p[int(k)] = v
    r = oracle.peaks(p, geo)
    assert r["n"] == len(case["expect"])
    for i, e in enumerate(case["expect"]):
        assert r["t"][i] == e["t"]
        assert r["z"][i] == pytest.approx(e["z"], rel=1e-15, abs=1e-13)
        assert r["prob"][i] == e["prob"]
        assert r["integral"][i] == pytest.approx(e["integral"], rel=1e-15)


def test_local_maxima_match_scipy():
    """Local-maximum step vs scipy.signal.find_peaks with plateau_size=(1, 1)
    (single-sample peaks only, so plateaus are excluded) and an integral
    threshold below any window sum."""
    rng = np.random.default_rng(11)
    geo = oracle.Geometry(s_min=-1.0)
    for trial in range(20):
        p = rng.uniform(0, 1, 4000)
        if trial % 2:
            p = np.round(p * 8) / 8          # many exact ties and plateaus
        r = oracle.peaks(p, geo)
        ref, _ = find_peaks(p, height=0.01 + 1e-12, plateau_size=(1, 1))
        ref = ref[p[ref] > 0.01]
        assert np.array_equal(r["t"], ref)


def test_window_sums_and_centroids_vs_numpy():
    rng = np.random.default_rng(12)
    p = rng.uniform(0, 1, 4000)
    geo = oracle.Geometry()
    r = oracle.peaks(p, geo)
    zc = -100.0 + 0.1 * (np.arange(4000) + 0.5)
    for i in range(0, len(r["t"]), 37):
        t = r["t"][i]
        lo, hi = max(0, t - 5), min(3999, t + 5)
        S = p[lo:hi + 1].sum()
        assert r["integral"][i] == pytest.approx(S, rel=1e-14)
        assert r["z"][i] == pytest.approx((p[lo:hi + 1] * zc[lo:hi + 1]).sum() / S, rel=1e-13)
        assert r["prob"][i] == p[t]


def test_gaussian_bumps_land_on_their_centres():
    """Hand-built probability: sums of narrow Gaussians centred on bin centres;
    each vertex is found at its bin and, being symmetric and isolated, its
    centroid is that bin's centre."""
    L = 4000
    t = np.arange(L)
    centres = [150, 700, 1333, 2500, 3801]
    p = np.zeros(L)
    for c in centres:
        p += 0.6 * np.exp(-0.5 * ((t - c) / 1.5) ** 2)
    r = oracle.peaks(p, oracle.Geometry())
    assert list(r["t"]) == centres
    np.testing.assert_allclose(r["z"], -100.0 + 0.1 * (np.array(centres) + 0.5), rtol=0, atol=1e-12)


def test_truncation_reports_the_full_count():
    p = np.tile([0.1, 0.9], 2000)
    geo = oracle.Geometry(max_peaks=10)
    r = oracle.peaks(p, geo)
    assert r["n"] == 1999 and len(r["t"]) == 10
