"""GPU parity of the FP32 HIP path against the FP64 oracle, through the C ABI.

Workloads (seeded, synthetic, see synth/): the 8-event parity batch
(Poisson(180) tracks, Poisson(5.6) vertices), the 1000-event production
batch, and heavy-tailed batches (log-normal track counts up to 1500).
Bars (tests/parity.py): p within 1e-4 relative, identical peak sets on every
robust decision, histogram exact where it is zero, and every event's vertex
list index-exact against the oracle's peak finder run on the GPU's own p.
"""

import numpy as np
import pytest

import oracle
from synth import make_events
from synth.events import pack_events
from tests import parity
from tests.gpu_util import torch_cuda, make_engine, run, geometry, event_vertices, weights

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-parity]", *a, flush=True)


@pytest.fixture(scope="module")
def eng8():
    torch_cuda()
    say("engine max_events=8")
    e = make_engine(8)
    yield e
    e.close()


@pytest.fixture(scope="module")
def batch8():
    return make_events(8, seed=0)


@pytest.fixture(scope="module")
def ref8(batch8):
    return oracle.run_batch(batch8, weights())


@pytest.fixture(scope="module")
def out8(eng8, batch8):
    say("execute 8-event batch")
    return run(eng8, batch8)


def test_probability_parity(out8, ref8):
    errs = [parity.max_rel(out8["prob"][e], ref8[e]["p"]) for e in range(8)]
    say("max rel err p per event", ["%.2e" % x for x in errs])
    assert max(errs) <= parity.P_REL


def test_peak_parity(eng8, out8, ref8):
    geo = geometry(eng8)
    total_amb = 0
    for e in range(8):
        bins, z, h, S = event_vertices(out8, e)
        assert out8["n_vertices"][e] == len(bins)
        amb, n = parity.compare_peaks(bins, z, h, S, ref8[e], geo)
        total_amb += amb
    say("ambiguous decisions excluded:", total_amb)
    assert total_amb < 100
    nv = parity.exact_peaks_all(out8, geo)
    say(f"exact peaks on the GPU's p: {nv} vertices, no exclusions")


def test_status_ok(out8, ref8):
    assert np.all(out8["status"] == 0)


def test_histogram_parity(eng8, out8, ref8):
    hist = eng8.debug_tensor("hist", 8).cpu().numpy().reshape(8, -1)
    s_in = weights().s_in
    for e in range(8):
        ref = s_in * ref8[e]["H"]
        nz = ref != 0
        assert np.all(hist[e][~nz] == 0)
        assert parity.max_rel(hist[e][nz], ref[nz]) <= parity.P_REL


@pytest.fixture(scope="module")
def eng_seeds():
    # an engine of its own: the layer tests below read eng8's stored
    # activations of the seed-0 batch
    torch_cuda()
    e = make_engine(8)
    yield e
    e.close()


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_parity_other_seeds(eng_seeds, seed):
    """p, histogram and peaks of three more 8-event batches (other event
    streams of the same generator) against the oracle, at the same bars."""
    eng = eng_seeds
    batch = make_events(8, seed=seed)
    ref = oracle.run_batch(batch, weights())
    say(f"execute 8-event batch of seed {seed}")
    out = run(eng, batch)
    errs = [parity.max_rel(out["prob"][e], ref[e]["p"]) for e in range(8)]
    say(f"seed {seed}: max rel err p %.2e" % max(errs))
    assert max(errs) <= parity.P_REL
    hist = eng.debug_tensor("hist", 8).cpu().numpy().reshape(8, -1)
    s_in = weights().s_in
    geo = geometry(eng)
    total_amb = 0
    for e in range(8):
        h_ref = s_in * ref[e]["H"]
        nz = h_ref != 0
        assert np.all(hist[e][~nz] == 0)
        assert parity.max_rel(hist[e][nz], h_ref[nz]) <= parity.P_REL
        bins, z, hh, S = event_vertices(out, e)
        assert out["n_vertices"][e] == len(bins)
        amb, _ = parity.compare_peaks(bins, z, hh, S, ref[e], geo)
        total_amb += amb
    say(f"seed {seed}: ambiguous decisions excluded:", total_amb)
    assert total_amb < 100
    parity.exact_peaks_all(out, geo)


LAYERS = ["enc0.c2", "pool0", "enc1.c2", "pool1", "enc2.c2", "pool2", "enc3.c1", "enc3.c2",
          "up2", "dec2.c1", "dec2.c2", "up1", "dec1.c1", "dec1.c2", "up0", "dec0.c1"]


@pytest.mark.parametrize("name", LAYERS)
def test_layer_parity(eng8, batch8, out8, name):
    """Every stored activation of event 0 against the oracle's taps."""
    w = weights()
    ref = oracle.unet_taps(w.s_in * oracle.histogram(batch8.tracks_of(0), w)[0], w)[name]
    got = eng8.debug_tensor(name, 1).cpu().numpy().reshape(ref.shape)
    err = parity.tap_err(got, ref)
    say(name, "normwise tap err %.2e" % err)
    assert err <= parity.TAP_NORM


def test_deterministic_rerun(eng8, batch8, out8):
    again = run(eng8, batch8)
    for k in ("prob", "z", "integral", "n_vertices", "bin"):
        assert np.array_equal(again[k], out8[k]), k


def test_batch_invariance(eng8, batch8, out8):
    """An event alone gives the same bits as inside the batch."""
    for e in (0, 5):
        alone = run(eng8, batch8.subset([e]))
        assert np.array_equal(alone["prob"][0], out8["prob"][e])
        n = out8["n_vertices"][e]
        assert alone["n_vertices"][0] == n
        assert np.array_equal(alone["z"][0, :n], out8["z"][e, :n])


def test_track_order_invariance(eng8, batch8, out8):
    tr = batch8.tracks_of(2)
    perm = np.random.default_rng(3).permutation(tr.shape[1])
    out = run(eng8, pack_events([tr[:, perm]]))
    assert parity.max_rel(out["prob"][0], out8["prob"][2]) <= 1e-5


def test_edge_events(eng8):
    """Zero tracks, one track, out-of-window and non-finite tracks, an event
    over the track cap, and decreasing offsets (bypass) in one batch."""
    import paper_2602_19959_amd as pv
    torch = torch_cuda()
    ev = make_events(4, seed=5)
    t0 = ev.tracks_of(0).copy()
    t0[0, :3] = [-150.0, 300.0, np.nan]
    t0[5, 3] = np.inf
    one = ev.tracks_of(1)[:, :1].copy()
    lists = [np.zeros((9, 0), np.float32), one, t0, ev.tracks_of(3)]
    batch = pack_events(lists)
    say("edge batch")
    out = run(eng8, batch)
    w = weights()
    refs = [oracle.run_event(t, w) for t in lists]
    geo = geometry(eng8)
    for e in range(4):
        assert parity.max_rel(out["prob"][e], refs[e]["p"]) <= parity.P_REL, e
        bins, z, h, S = event_vertices(out, e)
        parity.compare_peaks(bins, z, h, S, refs[e], geo)
    parity.exact_peaks_all(out, geo)
    assert out["status"][0] == 0 and out["status"][1] == 0 and out["status"][3] == 0
    assert out["status"][2] == pv.EV_TRACKS_DROPPED
    # over the cap: bypassed, neighbours unchanged
    big = make_engine(4, max_tracks_per_event=50)
    res = run(big, batch)
    assert res["status"][2] & pv.EV_TOO_MANY_TRACKS and res["n_vertices"][2] == 0
    assert res["status"][3] & pv.EV_TOO_MANY_TRACKS
    assert res["status"][0] == 0 and np.array_equal(res["prob"][0], out["prob"][0])
    assert np.array_equal(res["prob"][1], out["prob"][1])
    parity.exact_peaks_all(res, geo)
    # decreasing offsets: bypass that event only
    feat, off = pv.upload_events(batch)
    bad = off.clone()
    bad[2] = bad[1] - 1                  # event 1 ends before it starts
    o = big.alloc_outputs(4)
    big.execute(feat, bad, o)
    big.synchronize()
    h = o.to_host()
    assert h["status"][1] & pv.EV_BAD_INPUT and h["n_vertices"][1] == 0
    assert np.array_equal(h["prob"][0], out["prob"][0]) and h["status"][0] == 0
    big.close()


@pytest.mark.parametrize("hw,s_min", [(0, 0.2), (3, 3.0), (5, 5.0), (8, 8.0)])
def test_peaks_other_windows(batch8, ref8, hw, s_min):
    """Other half-widths and window thresholds (the window test then rejects
    part of the local maxima); the oracle finds peaks on its own p."""
    torch_cuda()
    eng = make_engine(8, half_window=hw, integral_min=s_min)
    out = run(eng, batch8)
    geo = geometry(eng)
    assert geo.half_window == hw and geo.s_min == s_min
    kept = 0
    for e in range(8):
        ref = dict(oracle.peaks(ref8[e]["p"], geo), p=ref8[e]["p"])
        bins, z, h, S = event_vertices(out, e)
        parity.compare_peaks(bins, z, h, S, ref, geo)
        kept += len(bins)
    assert parity.exact_peaks_all(out, geo) == kept
    say(f"hw {hw} s_min {s_min}: {kept} vertices")
    eng.close()


@pytest.mark.parametrize("dtype,n_bins", [("fp32", 16000), ("bf16", 16000), ("bf16", 4800)])
def test_longest_histogram(dtype, n_bins):
    """The longest histogram the spec takes with the paper's 100-bin
    intervals: 16000 bins (160 intervals; at most 16384 bins), so the UNet
    rows, the track stage's LDS histogram and the peak finder's row and
    candidate list are at their largest; in BF16 the matrix-core network
    then accumulates in LDS (more intervals than its register histogram
    holds).  4800 bins (48 intervals) is the register histogram's largest
    case.  p and peaks of two events against the oracle (FP32 at the FP32
    bar, BF16 within its stated bound)."""
    torch_cuda()
    eng = make_engine(2, n_bins=n_bins, max_peaks_per_event=n_bins // 2, compute_dtype=dtype)
    batch = make_events(2, seed=0)
    say(f"{n_bins}-bin engine", dtype, eng.launch_kernels()[0])
    assert eng.launch_kernels()[0].startswith("track_stage_mma<" if dtype != "fp32" and n_bins <= 4800
                                              else "track_stage_queue<")
    out = run(eng, batch)
    geo = geometry(eng)
    assert geo.n_bins == n_bins
    refs = oracle.run_batch(batch, weights(), geo)
    for e in range(2):
        ref = refs[e]
        assert ref["n"] < n_bins // 2
        if dtype == "fp32":
            assert parity.max_rel(out["prob"][e], ref["p"]) <= parity.P_REL, e
            bins, z, h, S = event_vertices(out, e)
            parity.compare_peaks(bins, z, h, S, ref, geo)
        else:
            assert float(np.max(np.abs(out["prob"][e] - ref["p"]))) <= parity.P_ABS[dtype], e
        assert out["status"][e] == 0
    parity.exact_peaks_all(out, geo)
    eng.close()


def test_first_conv_fused_and_standalone_agree(eng8, batch8, out8):
    """By default enc0.c2 computes the first convolution in its staging; with
    a tile variant that cannot (a double-buffered one) the standalone
    first-convolution kernel runs before it.  Both give the same bits."""
    names, kernels = eng8.launch_names(), eng8.launch_kernels()
    i = names.index("enc0.c2")
    assert names[i - 1] == "enc0.c1"
    assert kernels[i].startswith("conv_mfma_f32_first<") and kernels[i - 1] == "first_conv (in enc0.c2)"
    base = eng8.variants()[i]
    db = next(v for v in range(eng8.variant_count(i)) if eng8.set_variant(i, v) and "_db<" in eng8.launch_kernels()[i])
    try:
        assert eng8.launch_kernels()[i - 1] == "first_conv", db
        got = run(eng8, batch8)
        for k in ("prob", "z", "integral", "n_vertices", "bin"):
            assert np.array_equal(got[k], out8[k]), k
    finally:
        eng8.set_variant(i, base)
    assert eng8.launch_kernels()[i].startswith("conv_mfma_f32_first<")


@pytest.mark.parametrize("dtype", ["fp32", "bf16"])
def test_ragged_shapes(dtype):
    """A histogram of 3978 bins (39 intervals of 102) and a 2-level UNet: no
    row count is a multiple of a tile, the bottom level has an odd length
    (1989), the track network has 102 outputs and the peak finder's row is
    not a multiple of four floats.  p and peaks of four events against the
    oracle (FP32 at the FP32 bar, BF16 within its stated bound)."""
    from synth import NetShape
    torch_cuda()
    shape = NetShape(n_out=102, n_levels=2)
    eng = make_engine(4, shape=shape, n_bins=3978, bins_per_interval=102, compute_dtype=dtype,
                      max_peaks_per_event=3978)
    batch = make_events(4, seed=7)
    say("ragged engine", dtype)
    out = run(eng, batch)
    geo = geometry(eng)
    assert geo.n_bins == 3978 and geo.bins_per_interval == 102
    refs = oracle.run_batch(batch, weights(0, shape), geo)
    for e in range(4):
        if dtype == "fp32":
            assert parity.max_rel(out["prob"][e], refs[e]["p"]) <= parity.P_REL, e
            bins, z, h, S = event_vertices(out, e)
            parity.compare_peaks(bins, z, h, S, refs[e], geo)
        else:
            assert float(np.max(np.abs(out["prob"][e] - refs[e]["p"]))) <= parity.P_ABS[dtype], e
        assert (out["status"][e] & ~pv_dropped()) == 0
    parity.exact_peaks_all(out, geo)
    eng.close()


@pytest.mark.parametrize("dtype", ["fp32", "bf16"])
@pytest.mark.parametrize("n_bins,bpi", [(800, 100), (400, 10)])
def test_short_histograms(dtype, n_bins, bpi):
    """Histograms inside one interval tile of the register histogram: 8
    intervals of 100 bins, and 40 intervals of 10 bins (one partly used
    column tile: three of the four waves hold no output columns), windows
    centred on the vertices.  p and peaks of four events against the oracle
    (FP32 at the FP32 bar, BF16 within its stated bound)."""
    from synth import NetShape
    torch_cuda()
    shape = NetShape(n_out=bpi)
    z_min = -0.05 * n_bins
    eng = make_engine(4, shape=shape, n_bins=n_bins, bins_per_interval=bpi, z_min_mm=z_min,
                      compute_dtype=dtype, max_peaks_per_event=n_bins // 2)
    assert eng.launch_kernels()[0].startswith("track_stage_mma<")
    batch = make_events(4, seed=9)
    say("short histogram", n_bins, bpi, dtype)
    out = run(eng, batch)
    geo = geometry(eng)
    assert geo.n_bins == n_bins and geo.bins_per_interval == bpi and geo.z_min == z_min
    refs = oracle.run_batch(batch, weights(0, shape), geo)
    for e in range(4):
        if dtype == "fp32":
            assert parity.max_rel(out["prob"][e], refs[e]["p"]) <= parity.P_REL, e
            bins, z, h, S = event_vertices(out, e)
            parity.compare_peaks(bins, z, h, S, refs[e], geo)
        else:
            assert float(np.max(np.abs(out["prob"][e] - refs[e]["p"]))) <= parity.P_ABS[dtype], e
        assert (out["status"][e] & ~pv_dropped()) == 0
    parity.exact_peaks_all(out, geo)
    eng.close()


def pv_dropped():
    import paper_2602_19959_amd as pv
    return pv.EV_TRACKS_DROPPED


def test_peak_truncation():
    import paper_2602_19959_amd as pv
    torch_cuda()
    e = make_engine(2, max_peaks_per_event=10)
    batch = make_events(2, seed=0)
    out = run(e, batch)
    w = weights()
    ref = oracle.run_event(batch.tracks_of(0), w)
    assert out["n_vertices"][0] == 10 and out["status"][0] & pv.EV_PEAKS_TRUNCATED
    assert np.array_equal(out["bin"][0, :10], ref["t"][:10])
    parity.exact_peaks_all(out, geometry(e))
    e.close()


def test_empty_batch(eng8):
    torch = torch_cuda()
    import paper_2602_19959_amd as pv
    feat = torch.zeros(9, 0, dtype=torch.float32, device="cuda")
    off = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = eng8.alloc_outputs(0)
    eng8.execute(feat, off, out)
    eng8.synchronize()


def test_capacity_errors(eng8, batch8):
    import paper_2602_19959_amd as pv
    torch = torch_cuda()
    big = make_events(9, seed=1)
    feat, off = pv.upload_events(big)
    with pytest.raises(pv.PvfError) as ei:
        eng8.execute(feat, off, eng8.alloc_outputs(9))
    assert ei.value.status == 3


def test_every_variant_gives_identical_bits(eng8, batch8, out8):
    """Tile-shape variants only change speed: each one reproduces the
    default configuration's outputs bit for bit, and the autotuner's pick
    does too."""
    base = eng8.variants()
    n = len(base)
    tried = 0
    for v in range(eng8.variant_count(2)):
        changed = [i for i in range(n) if base[i] >= 0 and eng8.set_variant(i, v)]
        if not changed:
            continue
        tried += 1
        say(f"variant {v} on launches {changed}")
        got = run(eng8, batch8)
        for k in ("prob", "z", "integral", "n_vertices", "bin"):
            assert np.array_equal(got[k], out8[k]), (v, k)
        for i in range(n):
            if base[i] >= 0:
                eng8.set_variant(i, base[i])
    assert tried >= 8
    import paper_2602_19959_amd as pv
    feat, off = pv.upload_events(batch8)
    picked = eng8.autotune(feat, off, reps=1)
    say("autotuned variants", picked)
    got = run(eng8, batch8)
    assert np.array_equal(got["prob"], out8["prob"])
    for i in range(n):
        if base[i] >= 0:
            eng8.set_variant(i, base[i])
