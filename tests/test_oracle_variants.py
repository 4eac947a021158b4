"""Pins of the oracle's Section 3 variants: boundary tracks feeding a second
interval, and the interval-batched UNet layout.

What fixes the answers here, independently of the oracle's code:
  * softplus outputs are strictly positive, so the intervals a track touches
    are exactly the intervals whose bins are non-zero; the boundary rule
    (strict distance to a shared edge, never across the ends of the
    histogram) is re-derived below from the edge positions alone;
  * the neighbour's frame is continuous with its own: a track just inside
    interval i seen from interval i-1 is the same input as a track just
    inside interval i-1 seen from its own interval, up to the distance moved;
  * moving an event by exactly one interval moves its histogram by one
    interval, bit for bit, away from the histogram's ends;
  * with one interval the two UNet layouts are the same computation, and in
    the interval layout no interval sees another's bins.
"""

import dataclasses

import numpy as np
import pytest

import oracle
from synth import make_weights

W = make_weights(0)
GEO = oracle.Geometry()
I_MM = GEO.interval_mm          # 10 mm


def track(z, seed=0):
    """One track at z with seeded other features (float32 [9][1])."""
    rng = np.random.default_rng(seed)
    f = np.zeros((9, 1), np.float32)
    f[0, 0] = z
    f[1:3, 0] = rng.normal(0, 0.05, 2)
    f[3:6, 0] = rng.normal(0, 0.3, 3)
    f[6:9, 0] = np.abs(rng.normal(0.05, 0.02, 3))
    return f


def support(H, geo=GEO):
    """Intervals whose bins are all non-zero (and the rest must be all zero)."""
    Hi = H.reshape(geo.n_intervals, geo.bins_per_interval)
    on = [i for i in range(geo.n_intervals) if np.all(Hi[i] > 0)]
    off = [i for i in range(geo.n_intervals) if i not in on]
    assert np.all(Hi[off] == 0)
    return on


def expected_intervals(z, b, geo=GEO):
    """The rule from the edge positions alone (double arithmetic, as in binning)."""
    z = float(np.float32(z))
    i = int(np.floor((z - geo.z_min) / geo.interval_mm))
    if not 0 <= i < geo.n_intervals:
        return []
    lo = geo.z_min + geo.interval_mm * i
    hi = geo.z_min + geo.interval_mm * (i + 1)
    out = [i]
    if b > 0 and z - lo < b and i > 0:
        out.append(i - 1)
    elif b > 0 and hi - z < b and i < geo.n_intervals - 1:
        out.append(i + 1)
    return sorted(out)


@pytest.mark.parametrize("z,b", [
    (-55.0, 1.0), (-59.5, 1.0), (-50.25, 1.0), (-50.0 - 2 ** -10, 1.0),
    (-50.0, 1.0), (-49.0, 1.0), (-49.0 + 2 ** -10, 1.0), (-51.0, 1.0), (-51.0 - 2 ** -10, 1.0),
    (-100.0, 2.0), (-99.5, 2.0), (299.5, 2.0), (299.0, 0.5), (5.0, 5.0), (4.999, 5.0), (0.001, 5.0),
    (12.0, 0.0), (19.9, 0.0),
])
def test_boundary_rule_sets_the_touched_intervals(z, b):
    geo = dataclasses.replace(GEO, boundary_mm=b)
    H, dropped = oracle.histogram(track(z), W, geo)
    assert dropped == 0
    assert support(H, geo) == expected_intervals(z, b, geo)


def test_no_boundary_equals_one_interval_histogram():
    rng = np.random.default_rng(3)
    f = np.stack([track(z, k)[:, 0] for k, z in enumerate(rng.uniform(-100, 300, 200))], axis=1)
    H0, _ = oracle.histogram(f, W)
    H1, _ = oracle.histogram(f, W, dataclasses.replace(GEO, boundary_mm=0.0))
    assert np.array_equal(H0, H1)


def test_boundary_adds_exactly_the_neighbour_terms():
    """With b > 0 the histogram is the one-interval histogram plus, per
    boundary track, one extra 100-bin block; tracks away from every edge
    change nothing."""
    geo = dataclasses.replace(GEO, boundary_mm=1.0)
    zs = [-72.5, -75.0, 13.3, 288.8]                 # all >= 1 mm from every edge
    f = np.stack([track(z, k)[:, 0] for k, z in enumerate(zs)], axis=1)
    assert np.array_equal(oracle.histogram(f, W, geo)[0], oracle.histogram(f, W)[0])
    g = np.concatenate([f, track(-69.5, 9)], axis=1)  # 0.5 mm above the edge at -70
    d = oracle.histogram(g, W, geo)[0] - oracle.histogram(g, W)[0]
    assert support(d, geo) == [2]                     # interval [-80, -70)


@pytest.mark.parametrize("edge_i", [5, 23])
def test_neighbour_frame_is_continuous(edge_i):
    """The contribution a track just above the edge of interval i gives to
    interval i-1 matches the contribution of a track just below the edge (in
    interval i-1, its own frame), and likewise above/below the upper edge."""
    geo = dataclasses.replace(GEO, boundary_mm=1.0)
    B = GEO.bins_per_interval
    edge = GEO.z_min + I_MM * edge_i
    eps = 2.0 ** -12
    up = oracle.histogram(track(edge + eps, 1), W, geo)[0]       # own i, neighbour i-1
    dn = oracle.histogram(track(edge - eps, 1), W, geo)[0]       # own i-1, neighbour i
    nb_lo = up[(edge_i - 1) * B:edge_i * B]
    own_lo = dn[(edge_i - 1) * B:edge_i * B]
    nb_hi = dn[edge_i * B:(edge_i + 1) * B]
    own_hi = up[edge_i * B:(edge_i + 1) * B]
    scale = np.max(np.abs(own_lo))
    assert np.max(np.abs(nb_lo - own_lo)) < 1e-3 * scale
    assert np.max(np.abs(nb_hi - own_hi)) < 1e-3 * scale
    # and the neighbour frame is not the own frame: a track at the bottom of
    # interval i seen from its own frame gives a clearly different block
    assert np.max(np.abs(nb_lo - own_hi)) > 1e-2 * scale


def test_shift_by_one_interval_is_exact():
    geo = dataclasses.replace(GEO, boundary_mm=1.5)
    B = GEO.bins_per_interval
    zs = [-60.0 + 0.25, -60.0 + 9.875, -55.0, -50.0 + 0.5, -41.0 - 0.125]
    f = np.stack([track(z, k)[:, 0] for k, z in enumerate(zs)], axis=1)
    g = f.copy()
    g[0] += np.float32(I_MM)
    assert np.array_equal(g[0] - f[0], np.full(len(zs), I_MM, np.float32))
    H1 = oracle.histogram(f, W, geo)[0]
    H2 = oracle.histogram(g, W, geo)[0]
    assert np.array_equal(H2[B:], H1[:-B])
    assert np.all(H2[:B] == 0)


def test_neighbour_helper_matches_rule():
    geo = dataclasses.replace(GEO, boundary_mm=0.75)
    for z in np.linspace(-99.99, 299.99, 4001):
        i = oracle.bin_index(z, geo)
        exp = [x for x in expected_intervals(z, 0.75, geo) if x != i]
        assert oracle.neighbour(z, i, geo) == (exp[0] if exp else -1)


# ---------------------------------------------------------------- layout

W3 = make_weights(0, shape=make_weights(0).shape.__class__(n_levels=3))


def test_interval_layout_single_interval_equals_event_layout():
    geo1 = oracle.Geometry(n_intervals=1, max_peaks=50)
    f = np.stack([track(-100 + z, k)[:, 0] for k, z in enumerate([1.0, 2.5, 2.6, 7.25])], axis=1)
    a = oracle.run_event(f, W3, geo1)
    b = oracle.run_event(f, W3, dataclasses.replace(geo1, layout="interval"))
    assert np.array_equal(a["logit"], b["logit"]) and a["n"] == b["n"]


def test_interval_layout_sees_no_other_interval():
    """All tracks in interval 7: in the interval layout every other interval
    sees a zero input (the same logits everywhere, the UNet of zeros), while
    the event layout lets interval 7's bins reach its neighbours."""
    geo = dataclasses.replace(GEO, layout="interval", max_peaks=200)
    B = GEO.bins_per_interval
    z7 = GEO.z_min + I_MM * 7
    f = np.stack([track(z7 + d, k)[:, 0] for k, d in enumerate([0.05, 3.0, 3.1, 9.95])], axis=1)
    r = oracle.run_event(f, W3, geo)
    lg = r["logit"].reshape(GEO.n_intervals, B)
    others = [i for i in range(GEO.n_intervals) if i != 7]
    for i in others:
        assert np.array_equal(lg[i], lg[0 if 7 != 0 else 1])
    zero = oracle.unet(np.zeros(B), W3)
    assert np.array_equal(lg[0], zero)
    assert np.array_equal(lg[7], oracle.unet(W3.s_in * r["H"][7 * B:8 * B], W3))
    ev = oracle.run_event(f, W3, dataclasses.replace(geo, layout="event"))
    le = ev["logit"].reshape(GEO.n_intervals, B)
    assert not np.array_equal(le[6], lg[6]) and not np.array_equal(le[8], lg[8])
    assert np.array_equal(le[2], le[3])           # far from interval 7 and the ends: the zero response
