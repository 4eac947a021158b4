"""The whole oracle path on the 8-event parity workload (seed 0) against an
independent float64 PyTorch restatement of the same network."""

import numpy as np
import pytest
import torch

import oracle
from synth import make_events, make_weights
from tests import torch_ref


@pytest.fixture(scope="module")
def run8():
    ev = make_events(8, seed=0)
    w = make_weights(0)
    return ev, w, oracle.run_batch(ev, w)


def test_forward_vs_torch_restatement(run8):
    ev, w, res = run8
    H = np.stack([torch_ref.histogram(ev.tracks_of(e), w).numpy() for e in range(8)])
    logit = torch_ref.unet(w.s_in * H, w).numpy()
    for e in range(8):
        np.testing.assert_allclose(res[e]["H"], H[e], rtol=1e-12, atol=0)
        np.testing.assert_allclose(res[e]["logit"], logit[e], rtol=1e-10, atol=1e-11)
        p = torch.sigmoid(torch.from_numpy(logit[e])).numpy()
        np.testing.assert_allclose(res[e]["p"], p, rtol=1e-12)


def test_forward_conditioning(run8):
    """The input scale keeps the network out of sigmoid saturation and the
    histogram carries the expected mass."""
    ev, w, res = run8
    lg = np.stack([r["logit"] for r in res])
    assert np.abs(lg).max() < 12
    for e, r in enumerate(res):
        assert r["dropped"] == 0
        assert 0 < r["n"] <= 1999
        assert np.all(np.diff(r["t"]) >= 2)          # strict maxima cannot touch


def test_batch_threads_do_not_change_results(run8):
    ev, w, res = run8
    one = oracle.run_batch(ev.subset([3, 5]), w, threads=1)
    for k, e in enumerate((3, 5)):
        assert np.array_equal(one[k]["p"], res[e]["p"])
        assert np.array_equal(one[k]["z"], res[e]["z"])
