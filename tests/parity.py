"""Comparison rules between the HIP path and the FP64 oracle.

Floating point:
* per-bin probability p: max relative error <= 1e-4 (the FP32 bar);
* histogram (scaled): relative error <= 1e-4 where the oracle is non-zero,
  exactly 0 where it is 0 (intervals without tracks);
* intermediate activations (used to localise a faulty layer, not the
  parity target): normwise, max|diff| / max|ref| <= 1e-5 per tensor.  A conv
  output is a sum of up to 1280 products and carries the rounding of every
  layer before it, so its FP32 error is absolute at the scale of the
  tensor's largest values (measured about 1e-6 of max|ref| at the deepest
  decoder layer); a wrong index or operand gives errors of order 1.

Peak set ("identical peaks"): every vertex decision is a conjunction of
three margins taken on the oracle's FP64 values -- the local-maximum margin
m1 = min(p[t]-p[t-1], p[t]-p[t+1]), the height margin m2 = p[t] - p_min and
the window margin m3 = S_t - s_min.  A decision is robust when no change of
the p values by less than delta/2 each can flip it (m1, m2 beyond delta, m3
beyond 11*delta, the window's bin count); the GPU must agree with the oracle
on every robust decision.  Non-robust ("ambiguous") bins are excluded and
counted.  delta = 1e-5 is ten times the FP32 path's worst absolute error on
p seen at the 8-event workload and ten times below the tolerance on p.
Matched vertices: |dz| <= 1e-4 mm, window sum and height within 1e-4 relative.
Ambiguous decisions are capped: outside the sigmoid's saturated range
(p_ref > 1 - SAT_EPS, where neighbouring probabilities differ by less than
FP32 can resolve) at most AMB_MAX_FRAC of an event's decisions may be
ambiguous; saturated ones are counted and reported.

The peak finder itself is checked without exclusions by exact_peaks: the
oracle's peak finder run on the GPU's own float32 p (upcast to double, which
is exact) must give the GPU's vertex list index for index.  Peak finding is
index work, so the bar there is bit-exact: the same bins, heights and window
sums (both sides add the same doubles in ascending bin order), the same
count and truncation flag, and z within 1e-12 relative (the centroid's
products may be fused on the GPU).
"""

import numpy as np

import oracle

P_REL = 1e-4
TAP_NORM = 1e-5
DELTA = 1e-5
Z_ABS = 1e-4
SAT_EPS = 1e-3
AMB_MAX_FRAC = 5e-3
Z_EXACT_REL = 1e-12


def max_rel(a, ref):
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.max(np.abs(a - ref) / np.abs(ref))) if ref.size else 0.0


def tap_err(a, ref):
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.max(np.abs(a - ref)) / np.max(np.abs(ref)))


def classify(p, geo):
    """Oracle decisions per bin: +1 robust vertex, -1 robust non-vertex, 0 ambiguous."""
    L = p.shape[0]
    out = -np.ones(L, np.int8)
    hw = geo.half_window
    cs = np.concatenate([[0.0], np.cumsum(p)])
    for t in range(1, L - 1):
        m1 = min(p[t] - p[t - 1], p[t] - p[t + 1])
        m2 = p[t] - geo.p_min
        lo, hi = max(0, t - hw), min(L - 1, t + hw)
        m3 = (cs[hi + 1] - cs[lo]) - geo.s_min
        width = hi - lo + 1
        if m1 >= DELTA and m2 >= DELTA and m3 >= width * DELTA:
            out[t] = 1
        elif m1 <= -DELTA or m2 <= -DELTA or m3 <= -width * DELTA:
            out[t] = -1
        else:
            out[t] = 0
    out[0] = out[L - 1] = -1
    return out


def ambiguity(ref, geo):
    """(ambiguous bins, of which saturated, decisions) of one oracle event;
    asserts the cap on the unsaturated ones."""
    cls = classify(ref["p"], geo)
    amb = np.nonzero(cls == 0)[0]
    sat = int(np.sum(ref["p"][amb] > 1.0 - SAT_EPS))
    n = max(int(ref["n"]), 1)
    assert len(amb) - sat <= AMB_MAX_FRAC * n, (len(amb), sat, n)
    return len(amb), sat, n


def exact_peaks(host, e, geo):
    """The GPU's vertex list of event e against the oracle's peak finder on
    the GPU's own p: no exclusions, index-exact.  Returns the vertex count."""
    p = np.asarray(host["prob"][e], np.float32).astype(np.float64)
    ref = oracle.peaks(p, geo)
    n = int(host["n_vertices"][e])
    status = int(host["status"][e])
    if status & 3:                        # bypassed event: no vertices at all
        assert n == 0
        return 0
    assert n == min(ref["n"], geo.max_peaks), (e, n, ref["n"])
    assert bool(status & 4) == (ref["n"] > geo.max_peaks), (e, status, ref["n"])
    bins = host["bin"][e, :n]
    assert np.array_equal(bins, ref["t"]), e
    assert np.array_equal(np.asarray(host["integral"][e, :n], np.float64), ref["integral"]), e
    assert np.array_equal(np.asarray(host["peak_prob"][e, :n], np.float32).astype(np.float64), ref["prob"]), e
    z = np.asarray(host["z"][e, :n], np.float64)
    assert np.all(np.abs(z - ref["z"]) <= Z_EXACT_REL * np.maximum(np.abs(ref["z"]), 1.0)), e
    return n


def exact_peaks_all(host, geo, events=None):
    """exact_peaks over every event (or the given ones); returns the total
    vertex count."""
    evs = range(len(host["n_vertices"])) if events is None else events
    return sum(exact_peaks(host, e, geo) for e in evs)


def compare_peaks(gpu_t, gpu_z, gpu_prob, gpu_S, ref, geo):
    """Check the GPU vertex list of one event against the oracle result dict.
    Returns (n_ambiguous, n_compared); raises AssertionError on a mismatch
    or when the ambiguous decisions outside saturation exceed the cap."""
    ambiguity(ref, geo)
    cls = classify(ref["p"], geo)
    gset = set(int(t) for t in gpu_t)
    rset = set(int(t) for t in ref["t"])
    amb = set(np.nonzero(cls == 0)[0].tolist())
    robust_yes = set(np.nonzero(cls == 1)[0].tolist())
    assert robust_yes <= rset, "classification disagrees with the oracle's own list"
    missing = (rset - amb) - gset
    extra = (gset - amb) - rset
    assert not missing and not extra, f"peak sets differ: missing {sorted(missing)[:10]}, extra {sorted(extra)[:10]}"
    ridx = {int(t): i for i, t in enumerate(ref["t"])}
    for k, t in enumerate(gpu_t):
        t = int(t)
        if t not in ridx:
            continue
        i = ridx[t]
        assert abs(gpu_z[k] - ref["z"][i]) <= Z_ABS, (t, gpu_z[k], ref["z"][i])
        assert abs(gpu_S[k] - ref["integral"][i]) <= P_REL * ref["integral"][i]
        assert abs(gpu_prob[k] - ref["prob"][i]) <= P_REL * ref["prob"][i]
    return len(amb), len(rset | gset)


# Reduced-precision paths (BF16/FP16 storage and weights, FP32 accumulation;
# FP8 e4m3 with per-channel calibration scales): max |p - p_ref| <= P_ABS,
# and vertices matched one-to-one within |dz| <= DZ_MATCH: at least
# MATCH_MIN of the oracle's, at most EXTRA_MAX (a fraction of the oracle's
# count) unmatched extras.  Each bound is derived, in
# tests/test_precision_bounds.py, from the CPU emulation of the rounding in
# tests/emulate.py against the oracle, and must sit between 1.15x and 4x the
# emulated maximum.  Emulated on the 16 seed-0 events: max|dp| 1.54e-2 (BF16),
# 1.58e-3 (FP16), 0.253 (FP8; calibration from 64 events of seed 5); matched
# 99.86%, 99.98%, 97.8%; extra 0.16%, 0.02%, 2.7%.  FP8's three mantissa bits
# (unit roundoff 2^-4 per stored value, compounded over 17 layers) set its
# bound.
P_ABS = {"bf16": 2e-2, "fp16": 5e-3, "fp8_e4m3": 0.3}
MATCH_MIN = {"bf16": 0.995, "fp16": 0.999, "fp8_e4m3": 0.95}
EXTRA_MAX = {"bf16": 0.005, "fp16": 0.001, "fp8_e4m3": 0.05}
DZ_MATCH = 0.05

# The 64-channel network (the paper's deployed width) sums twice as many
# rounded products per output and has larger activations; emulated on 6
# seed-1 events: max|dp| 3.5e-2 (BF16), 3.8e-3 (FP16), 0.40 (FP8), with
# 99.8-100% of vertices matched.
P_ABS_WIDE = {"bf16": 5e-2, "fp16": 7e-3, "fp8_e4m3": 0.5}
MATCH_MIN_WIDE = {"bf16": 0.995, "fp16": 0.999, "fp8_e4m3": 0.97}

# Heavy-tailed batches (log-normal track counts up to 1500): events of
# 1000-1500 tracks drive the logits beyond 100, and the deep layers' absolute
# rounding error with them; emulated BF16 over the 176 events of the
# 4096-event batch with at least 1000 tracks or sampled by the GPU test:
# max|dp| 0.176 (median 0.033).
P_ABS_HEAVY = {"bf16": 0.22}
MATCH_MIN_HEAVY = {"bf16": 0.95}


def match_vertices(z_gpu, z_ref, tol=DZ_MATCH):
    """One-to-one matching of two sorted vertex lists by |dz| <= tol
    (two-pointer sweep).  Returns the number of matched pairs."""
    a = np.sort(np.asarray(z_gpu, np.float64))
    b = np.sort(np.asarray(z_ref, np.float64))
    i = j = m = 0
    while i < len(a) and j < len(b):
        d = a[i] - b[j]
        if abs(d) <= tol:
            m += 1
            i += 1
            j += 1
        elif d < 0:
            i += 1
        else:
            j += 1
    return m
