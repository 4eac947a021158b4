"""FP8 (OCP e4m3) UNet on the matrix cores against the FP64 oracle, through
the C ABI.  Activations carry one scale per channel from a calibration batch
of other events; each convolution folds its input scales into its weights and
quantises every output column with its own scale (per-output-channel).  This
takes the paper's low-precision roadmap (Section 5) one format below FP16; the
bounds and their derivation are in tests/parity.py."""

import numpy as np
import pytest

import oracle
from synth import make_events
from tests import parity
from tests.gpu_util import torch_cuda, make_engine, run, weights, fp8_calibration, geometry

pytestmark = pytest.mark.gpu
DT = "fp8_e4m3"


def say(*a):
    print("[gpu-fp8]", *a, flush=True)


@pytest.fixture(scope="module")
def batch16():
    return make_events(16, seed=0)


@pytest.fixture(scope="module")
def ref16(batch16):
    return oracle.run_batch(batch16, weights())


@pytest.fixture(scope="module")
def amax():
    torch_cuda()
    say("calibration: FP32 engine, 64 events of seed 5")
    return fp8_calibration()


@pytest.fixture(scope="module")
def fp8(batch16, amax):
    say("engine fp8")
    eng = make_engine(16, fp8_amax=amax, compute_dtype=DT)
    out = run(eng, batch16)
    yield eng, out
    eng.close()


def test_calibration_table_matches_oracle_taps():
    """The table holds, per stored tensor and channel, the absolute maximum
    over the calibration batch: check two tensors against the oracle's
    per-layer activations of the same events."""
    torch_cuda()
    w = weights()
    batch = make_events(8, seed=5)
    amax = fp8_calibration(n_events=8, seed=5)
    eng = make_engine(8)
    names = eng.launch_names()
    eng.close()
    # stored tensors in launch order, with their channel counts
    stored = [n for n in names if n not in ("track", "peaks", "dec0.c2+head")]
    chans = {n: (32 << int(n[3])) if n.startswith(("enc", "dec")) else (32 << int(n[2])) for n in stored}
    n_unet = sum(chans.values())
    n_mlp = 9 + w.shape.n_hidden * w.shape.hidden         # every track-network layer input
    assert len(amax) == n_unet + n_mlp
    # the network's first inputs are the features of every kept track
    g_max = np.zeros(9)
    for e in range(batch.n_events):
        tr = batch.tracks_of(e)
        for t in range(tr.shape[1]):
            i = oracle.bin_index(tr[0, t])
            if i >= 0:
                g_max = np.maximum(g_max, np.abs(oracle.features(tr[:, t], i, w)))
    got = amax[n_unet:n_unet + 9]
    err = float(np.max(np.abs(got - g_max) / g_max))
    say("network inputs calibration max rel err %.2e" % err)
    assert err <= 1e-6
    off = {}
    k = 0
    for n in stored:
        off[n] = k
        k += chans[n]
    want = {n: np.zeros(chans[n]) for n in ("enc0.c1", "dec1.c2")}
    for e in range(batch.n_events):
        taps = oracle.unet_taps(w.s_in * oracle.histogram(batch.tracks_of(e), w)[0], w)
        for n in want:
            want[n] = np.maximum(want[n], np.abs(taps[n]).max(axis=1))
    for n, v in want.items():
        got = amax[off[n]:off[n] + chans[n]]
        err = float(np.max(np.abs(got - v) / np.maximum(v, 1e-30)))
        say(n, "calibration max rel err %.2e" % err)
        assert err <= 1e-4, n


@pytest.mark.parametrize("dtype", ["fp32", "bf16"])
def test_calibration_network_layers_count_kept_tracks(dtype):
    """The track network's entries of the calibration table: per layer input
    and channel, the largest |value| over the kept tracks only.  Two events
    of one kept track (and one out of the window) leave 255 padding rows in
    their 256-track chunk; with every network bias at +1 the padding rows'
    bias-only activations exceed the kept track's in several channels, and
    they must not count.  FP32 against an FP64 evaluation of the layers at
    1e-5 per channel; the BF16 network (16-bit layer inputs, six layers deep)
    within 3e-2 of each layer's largest entry, and below 1.5 times the kept
    maximum wherever the padding rows' value is over twice it."""
    import dataclasses
    import paper_2602_19959_amd as pv
    from synth import weights_to_blob
    from synth.events import pack_events
    torch_cuda()
    w0 = weights()
    t = dict(w0.tensors)
    for l in range(w0.shape.n_hidden):
        t[f"mlp{l}.b"] = np.full_like(t[f"mlp{l}.b"], 1.0)
    w = dataclasses.replace(w0, tensors=t)
    src = make_events(2, seed=11)
    lists = []
    for e in range(2):
        tr = src.tracks_of(e)[:, :2].copy()
        tr[0, 1] = 400.0                      # outside the histogram window: dropped
        lists.append(tr)
    batch = pack_events(lists)
    spec = pv.default_spec(max_events=2, max_tracks_total=16, compute_dtype=dtype)
    eng = pv.Engine(weights_to_blob(w), spec)
    feat, off = pv.upload_events(batch)
    amax = eng.calibrate(feat, off)
    eng.close()
    s = w.shape
    n_mlp = s.n_feat + s.n_hidden * s.hidden
    got = amax[len(amax) - n_mlp:]
    g = []
    for tr in lists:
        for k in range(tr.shape[1]):
            i = oracle.bin_index(tr[0, k])
            if i >= 0:
                g.append(np.asarray(oracle.features(tr[:, k], i, w), np.float64))
    h = np.stack(g)
    assert len(h) == 2
    z = np.zeros((1, s.n_feat))                # a padding row: zero inputs
    kept, pad = [np.abs(h).max(axis=0)], [np.zeros(s.n_feat)]
    for l in range(s.n_hidden):
        W = np.asarray(w[f"mlp{l}.w"], np.float64)
        b = np.asarray(w[f"mlp{l}.b"], np.float64)
        y, yz = h @ W.T + b, z @ W.T + b
        h, z = np.where(y >= 0, y, w.leaky * y), np.where(yz >= 0, yz, w.leaky * yz)
        kept.append(np.abs(h).max(axis=0))
        pad.append(np.abs(z[0]))
    n_above = sum(int(np.sum(p > 2 * k)) for k, p in zip(kept, pad))
    assert n_above >= 3                        # the check below has channels to bite on
    if dtype == "fp32":
        want = np.concatenate(kept)
        err = float(np.max(np.abs(got - want) / np.maximum(want, 1e-30)))
        say(dtype, "network calibration max rel err %.2e" % err)
        assert err <= 1e-5
        return
    o = 0
    for l, (k, p) in enumerate(zip(kept, pad)):
        gl = got[o:o + len(k)]
        o += len(k)
        err = float(np.max(np.abs(gl - k)) / np.max(k))
        say(dtype, "layer input", l, "normwise err %.2e" % err)
        assert err <= 3e-2, l
        above = p > 2 * k
        assert np.all(gl[above] < 1.5 * k[above]), l


def test_probability_within_stated_bound(fp8, ref16):
    eng, out = fp8
    dp = max(float(np.max(np.abs(out["prob"][e] - ref16[e]["p"]))) for e in range(16))
    say("max |dp| %.3e (bound %.2f)" % (dp, parity.P_ABS[DT]))
    assert dp <= parity.P_ABS[DT]


def test_vertices_agree(fp8, ref16):
    eng, out = fp8
    matched = extra = total = 0
    for e in range(16):
        n = int(out["n_vertices"][e])
        m = parity.match_vertices(out["z"][e, :n], ref16[e]["z"])
        matched += m
        extra += n - m
        total += len(ref16[e]["z"])
    say(f"vertices matched {matched}/{total}, extra {extra}")
    assert matched >= parity.MATCH_MIN[DT] * total
    assert extra <= parity.EXTRA_MAX[DT] * total
    parity.exact_peaks_all(out, geometry(eng))


def test_deterministic_and_batch_invariant(fp8, batch16):
    eng, out = fp8
    again = run(eng, batch16)
    assert np.array_equal(again["prob"], out["prob"])
    alone = run(eng, batch16.subset([7]))
    assert np.array_equal(alone["prob"][0], out["prob"][7])


def test_variants_identical(fp8, batch16):
    eng, out = fp8
    base = eng.variants()
    tried = 0
    for v in range(eng.variant_count(2)):
        changed = [i for i in range(len(base)) if base[i] >= 0 and eng.set_variant(i, v)]
        if not changed:
            continue
        tried += 1
        got = run(eng, batch16)
        assert np.array_equal(got["prob"], out["prob"]), v
        for i in range(len(base)):
            if base[i] >= 0:
                eng.set_variant(i, base[i])
    assert tried >= 3


def test_fused_transposed_convs_identical(fp8, batch16):
    """By default dec2.c2 and dec1.c2 run up1 and up0 in their epilogues on
    their FP8 output tiles; with both convs on tiles that cannot (part of
    their channels) the transposed convs run as launches of their own and
    every output is the same bit for bit."""
    from paper_2602_19959_amd._binding import PvfError
    eng, out = fp8
    names, kernels = eng.launch_names(), eng.launch_kernels()
    prods = [names.index(p) for p in ("dec2.c2", "dec1.c2")]
    for l, i in zip((1, 0), prods):
        assert names[i + 1] == f"up{l}" and kernels[i + 1] == f"transposed conv (in {names[i]})"
        with pytest.raises(PvfError):
            eng.debug_tensor(names[i], 1)
    base = eng.variants()
    try:
        for i in prods:
            for v in range(eng.variant_count(i)):
                if eng.set_variant(i, v) and not eng.launch_kernels()[i + 1].startswith("transposed conv (in"):
                    break
            else:
                pytest.fail(f"no unfused variant for {names[i]}")
        got = run(eng, batch16)
        for k in ("prob", "z", "integral", "n_vertices", "status", "bin"):
            assert np.array_equal(got[k], out[k]), k
    finally:
        for i, v in enumerate(base):
            if v >= 0:
                eng.set_variant(i, v)
    assert eng.launch_kernels() == kernels


def test_first_conv_fused_and_standalone_agree(fp8, batch16):
    """By default enc0.c2 computes the first convolution in its staging (the
    standalone kernel's arithmetic and output scale); with a tile variant that
    cannot, the standalone first-convolution kernel runs before it, and every
    output is the same bit for bit."""
    eng, out = fp8
    names, kernels = eng.launch_names(), eng.launch_kernels()
    i = names.index("enc0.c2")
    assert names[i - 1] == "enc0.c1"
    assert kernels[i].startswith("conv_mfma_fp8x64_first<") and kernels[i - 1] == "first_conv (in enc0.c2)"
    base = eng.variants()[i]
    try:
        for v in range(eng.variant_count(i)):
            if eng.set_variant(i, v) and eng.launch_kernels()[i - 1] == "first_conv":
                break
        else:
            pytest.fail("no variant of enc0.c2 without the fused first convolution")
        say("enc0.c2 unfused:", eng.launch_kernels()[i])
        got = run(eng, batch16)
        for k in ("prob", "z", "integral", "n_vertices", "status", "bin"):
            assert np.array_equal(got[k], out[k]), k
    finally:
        eng.set_variant(i, base)
    assert eng.launch_kernels() == kernels


def test_fused_level0_identical(fp8, batch16):
    """Head-launch variants 20 and 21 compute dec0.c1 in the same kernel (its
    FP8 codes stay in LDS) and the dec0.c1 slot enqueues nothing: every output
    equals the two-launch path bit for bit, and the debug view refuses the
    unstored dec0.c1 while fused."""
    from paper_2602_19959_amd._binding import PvfError
    eng, out = fp8
    names = eng.launch_names()
    h = names.index("dec0.c2+head")
    base = eng.variants()
    assert base[h] == 20, "the fused 4-wave head is the default"
    try:
        assert eng.set_variant(h, 13)   # the two-launch path as the reference
        want = run(eng, batch16)
        assert eng.launch_kernels()[h - 1] != "conv (in dec0.c2+head)"
        for k in ("prob", "z", "integral", "n_vertices", "status", "bin"):
            assert np.array_equal(want[k], out[k]), k
        for v in (20, 21):
            assert eng.set_variant(h, v)
            k = eng.launch_kernels()
            assert k[h - 1] == "conv (in dec0.c2+head)" and k[h].startswith("conv_mfma_fp8x64_dec0<"), k[h - 1:h + 1]
            got = run(eng, batch16)
            for key in ("prob", "z", "integral", "n_vertices", "status", "bin"):
                assert np.array_equal(got[key], out[key]), (v, key)
            with pytest.raises(PvfError):
                eng.debug_tensor("dec0.c1", 1)
            say("fused level 0, variant", v, "identical")
    finally:
        for i, v in enumerate(base):
            if v >= 0:
                eng.set_variant(i, v)


def test_layer_taps_close_to_fp32(fp8, batch16):
    """Per-layer activations (dequantised with their channel scales) stay
    within FP8 rounding of the oracle's, normwise: 3 mantissa bits give a
    unit roundoff of 2^-4 per stored value, and each layer compounds the
    rounding of its inputs, weights and output."""
    eng, out = fp8
    w = weights()
    taps = oracle.unet_taps(w.s_in * oracle.histogram(batch16.tracks_of(0), w)[0], w)
    # event 0 alone, with the head on a tile that leaves dec0.c1 to its own
    # launch (the fused head keeps dec0.c1 in LDS)
    h = eng.launch_names().index("dec0.c2+head")
    vh = eng.variants()[h]
    assert eng.set_variant(h, 13)
    try:
        run(eng, batch16.subset([0]))
        for name, bound in (("enc0.c2", 0.08), ("pool1", 0.1), ("enc3.c2", 0.2),
                            ("up2", 0.2), ("dec1.c1", 0.2), ("dec0.c1", 0.25)):
            got = eng.debug_tensor(name, 1).cpu().numpy().reshape(taps[name].shape)
            err = parity.tap_err(got, taps[name])
            say(name, "normwise %.3e (bound %.2f)" % (err, bound))
            assert err <= bound, name
    finally:
        eng.set_variant(h, vh)


def test_full_batch_sampled(amax):
    """1000 events in one call, sampled against the oracle."""
    batch = make_events(1000, seed=0)
    eng = make_engine(1000, fp8_amax=amax, compute_dtype=DT)
    out = run(eng, batch)
    sample = [0, 333, 999]
    ref = oracle.run_batch(batch.subset(sample), weights())
    for k, e in enumerate(sample):
        dp = float(np.max(np.abs(out["prob"][e] - ref[k]["p"])))
        say(f"event {e} max |dp| {dp:.3e}")
        assert dp <= parity.P_ABS[DT]
    parity.exact_peaks_all(out, geometry(eng))
    eng.close()


def test_wrong_table_size_rejected(amax):
    import paper_2602_19959_amd as pv
    with pytest.raises(pv.PvfError):
        make_engine(4, fp8_amax=amax[:-1], compute_dtype=DT)
