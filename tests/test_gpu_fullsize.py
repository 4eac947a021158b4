"""Parity at the full batch sizes, in the launch configuration the benchmark
times: 1000 events (Poisson(180) tracks) and 4096 heavy-tailed events
(log-normal track counts, median 180, clipped to [5, 1500]).  The oracle
checks a sample of events one by one (first, last, largest, random); every
event's vertex list is checked index-exactly against the oracle's peak finder
on the GPU's own p; every sampled event's result must also equal, bit for
bit, that event run alone."""

import numpy as np
import pytest

import oracle
from synth import make_events
from tests import parity
from tests.gpu_util import torch_cuda, make_engine, run, geometry, event_vertices, weights

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-fullsize]", *a, flush=True)


@pytest.mark.parametrize("n_events,mix", [(1000, "poisson"), (4096, "lognormal")])
def test_full_batch_sampled(n_events, mix):
    torch_cuda()
    batch = make_events(n_events, seed=0, mix=mix)
    T = np.diff(batch.offsets)
    say(f"E={n_events} mix={mix} tracks total={T.sum()} max={T.max()}")
    eng = make_engine(n_events)
    out = run(eng, batch)
    assert np.all((out["status"] & 3) == 0)
    rng = np.random.default_rng(n_events)
    sample = sorted(set([0, n_events - 1, int(np.argmax(T)), int(np.argmin(T))] +
                        rng.choice(n_events, 4, replace=False).tolist()))
    ref = oracle.run_batch(batch.subset(sample), weights())
    geo = geometry(eng)
    for k, e in enumerate(sample):
        err = parity.max_rel(out["prob"][e], ref[k]["p"])
        bins, z, h, S = event_vertices(out, e)
        amb, sat, n = parity.ambiguity(ref[k], geo)
        parity.compare_peaks(bins, z, h, S, ref[k], geo)
        say(f"event {e} T={T[e]} max|logit| {np.abs(ref[k]['logit']).max():.1f} max rel {err:.2e} "
            f"vertices {n} ambiguous {amb} ({amb / n:.2%}; saturated {sat}, "
            f"other {amb - sat} <= {parity.AMB_MAX_FRAC:.1%} of {n})")
        assert err <= parity.P_REL
    nv = parity.exact_peaks_all(out, geo)
    say(f"exact peaks on the GPU's p, all {n_events} events: {nv} vertices, no exclusions")
    # batch invariance on the same sample
    alone_eng = make_engine(len(sample))
    alone = run(alone_eng, batch.subset(sample))
    for k, e in enumerate(sample):
        assert np.array_equal(alone["prob"][k], out["prob"][e])
    alone_eng.close()
    eng.close()
