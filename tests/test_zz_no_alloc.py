"""pvf_execute_scratch, the entry point for callers that cannot allocate:
the per-batch buffers live in the library's fixed per-device scratch.  Its
results must equal pvf_execute's bit for bit on two calls in a row, the
second with a smaller batch (so the second call's regions sit where the
first call left data, and its zero padding must be cleared again), and a
batch too large for the scratch is refused before anything is enqueued."""

import numpy as np
import pytest

from synth import NetShape, make_events
from tests.gpu_util import torch_cuda, engine_for, make_engine

pytestmark = pytest.mark.gpu

KEYS = ("prob", "z", "integral", "peak_prob", "n_vertices", "status", "bin")


def say(*a):
    print("[no-alloc]", *a, flush=True)


def run_both(eng, batch, with_prob):
    import paper_2602_19959_amd as pv
    feat, off = pv.upload_events(batch)
    ref = eng.alloc_outputs(batch.n_events, with_prob=with_prob)
    eng.execute(feat, off, ref)
    eng.synchronize()
    got = eng.alloc_outputs(batch.n_events, with_prob=with_prob)
    eng.execute_scratch(feat, off, got)
    eng.synchronize()
    return ref.to_host(), got.to_host()


def check_equal(ref, got, tag):
    for k in KEYS:
        if ref[k] is None:
            assert got[k] is None
            continue
        assert np.array_equal(ref[k], got[k]), (tag, k)


# (dtype, events of the first call, events of the second call, extra spec)
CASES = [
    ("fp32", 8, 3, {}),
    ("bf16", 16, 5, {}),
    ("fp8_e4m3", 32, 7, {}),
    ("fp32", 8, 2, {"unet_layout": "interval"}),     # 3-level network, 40 sequences per event
]
L3 = NetShape(n_levels=3)


@pytest.mark.parametrize("dtype,n1,n2,extra", CASES)
def test_scratch_matches_execute(dtype, n1, n2, extra):
    torch_cuda()
    say("case", dtype, n1, n2, extra)
    if extra:
        eng = make_engine(n1, shape=L3, compute_dtype=dtype, **extra)
    else:
        eng = engine_for(n1, dtype)
    first = make_events(n1, seed=11, mix="lognormal")
    second = make_events(n2, seed=12)
    ref, got = run_both(eng, first, with_prob=True)
    check_equal(ref, got, "first call")
    assert int(ref["n_vertices"].sum()) > 0
    say(dtype, "first call equal", n1, "events")
    # the second, smaller call: probabilities kept in the scratch too
    ref, got = run_both(eng, second, with_prob=False)
    check_equal(ref, got, "second call")
    say(dtype, "second call equal", n2, "events")
    eng.close()


def test_batch_too_large_for_scratch_is_refused():
    torch = torch_cuda()
    import paper_2602_19959_amd as pv
    from paper_2602_19959_amd._binding import PvfError
    say("case too large")
    eng = engine_for(12, "fp32")          # 12 FP32 events need about 86 MiB
    batch = make_events(12, seed=13)
    feat, off = pv.upload_events(batch)
    out = eng.alloc_outputs(12)
    with pytest.raises(PvfError) as ei:
        eng.execute_scratch(feat, off, out)
    assert ei.value.status == 9               # PVF_ERR_SCRATCH_TOO_SMALL
    eng.synchronize()
    h = out.to_host()
    assert not h["n_vertices"].any() and not h["prob"].any()   # nothing was enqueued
    # the engine still runs a batch that fits, and pvf_execute the large one
    ref, got = run_both(eng, make_events(6, seed=14), with_prob=True)
    check_equal(ref, got, "after refusal")
    eng.execute(feat, off, out)
    eng.synchronize()
    assert out.n_vertices.cpu().numpy().sum() > 0
    eng.close()
    del torch
