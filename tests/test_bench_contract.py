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
