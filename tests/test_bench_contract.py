"""bench.py's host-side contract, without a GPU: the error bounds it reports
are the ones the GPU tests enforce, its FLOP count is the UNet's closed form,
and more than one GPU is refused with a message."""

import os
import subprocess
import sys

import paper_2602_19959_amd as pv
from tests import parity

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_stated_tolerances_are_the_tested_ones():
    for dt, tol in bench.STATED_TOL.items():
        assert tol["max_abs_dp"] == parity.P_ABS[dt]
        assert tol["vertices_matched_min"] == parity.MATCH_MIN[dt]
        assert tol["extra_vertices_max"] == parity.EXTRA_MAX[dt]
    for dt, tol in bench.STATED_TOL_HEAVY.items():
        assert tol["max_abs_dp"] == parity.P_ABS_HEAVY[dt]
        assert tol["vertices_matched_min"] == parity.MATCH_MIN_HEAVY[dt]
        assert tol["extra_vertices_max"] == parity.EXTRA_MAX[dt]


def test_cpu_baseline_threads_follow_the_process_share(monkeypatch):
    """Every core of the affinity set, unless OMP_NUM_THREADS names a smaller
    share; the count and the share are reported."""
    aff = len(os.sched_getaffinity(0))
    monkeypatch.delenv("OMP_NUM_THREADS", raising=False)
    assert bench.cpu_threads() == (aff, aff, None)
    monkeypatch.setenv("OMP_NUM_THREADS", "1")
    assert bench.cpu_threads() == (1, aff, 1)
    monkeypatch.setenv("OMP_NUM_THREADS", str(aff + 100))
    assert bench.cpu_threads() == (aff, aff, aff + 100)


def test_native_oracle_build_gives_the_same_results(monkeypatch, tmp_path):
    """The CPU-baseline build for the host CPU (-march=native) computes the
    same numbers as the shipped build (no fast-math, no contraction)."""
    import numpy as np
    import oracle
    from synth import make_events, make_weights
    ev = make_events(1, seed=3)
    w = make_weights(0)
    ref = oracle.run_event(ev.tracks_of(0), w)
    monkeypatch.delenv("PVF_ORACLE_LIB", raising=False)
    flags = bench.native_oracle()
    assert "native" in flags
    lib = os.environ["PVF_ORACLE_LIB"]
    dst = str(tmp_path / "p.npy")
    code = ("import numpy as np, oracle; from synth import make_events, make_weights; "
            "r = oracle.run_event(make_events(1, seed=3).tracks_of(0), make_weights(0)); "
            f"np.save({dst!r}, r['p'])")
    subprocess.run([sys.executable, "-c", code], env=dict(os.environ, PVF_ORACLE_LIB=lib), cwd=ROOT,
                   capture_output=True, timeout=120, check=True)
    assert np.array_equal(np.load(dst), ref["p"])


def test_unet_flops_closed_form():
    """2 x sum over layers of L * Cout * Cin * taps, per event."""
    spec = pv.default_spec()
    macs = bench.layer_macs(spec)
    L, C = [4000 >> l for l in range(4)], [32 << l for l in range(4)]
    expect = 0
    for l in range(4):
        expect += L[l] * C[l] * (1 if l == 0 else C[l - 1]) * 5 + L[l] * C[l] * C[l] * 5
    for l in range(3):
        expect += L[l] * C[l] * 2 * C[l] + L[l] * C[l] * 2 * C[l] * 5 + L[l] * C[l] * C[l] * 5
    expect += L[0] * C[0]                      # 1x1 head
    got = sum(v for k, v in macs.items() if k not in ("track", "peaks"))
    assert got == expect
    assert abs(2 * got / 1e9 - 1.8775) < 1e-4
    # per track: 9x20 + 5 x 20x20 + 20x100 multiply-adds
    assert macs["track"] == 9 * 20 + 5 * 400 + 2000


def test_interval_layout_counts_every_interval():
    spec = pv.default_spec(unet_layout=1, n_levels=3)
    assert bench.units(spec) == 40
    per_seq = pv.default_spec(n_bins=100, n_levels=3)
    a = sum(v for k, v in bench.layer_macs(spec).items() if k not in ("track", "peaks"))
    b = sum(v for k, v in bench.layer_macs(per_seq).items() if k not in ("track", "peaks"))
    assert a == 40 * b


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
