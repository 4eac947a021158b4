"""The C ABI (include/pvf.h) without a GPU: the built library loads, exports
every declared symbol, its structs match the header byte for byte, and every
host-side validation answers before any device work.  Section 3 of the paper
asks for a frozen spec validated at init and a status code per call."""

import ctypes as C
import os
import subprocess
import textwrap

import pytest

import paper_2602_19959_amd as pv
from paper_2602_19959_amd import _binding as B
from synth import make_weights, weights_to_blob, NetShape

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_function():
    lib = pv.load_library()
    names = pv.declared_functions()
    assert "pvf_init" in names and "pvf_execute" in names and len(names) >= 10
    for n in names:
        assert hasattr(lib, n), f"{n} declared in pvf.h but not exported"


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(textwrap.dedent("""
        #include <stdio.h>
        #include <stddef.h>
        #include "pvf.h"
        int main(void) {
          printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(pvf_spec), offsetof(pvf_spec, max_tracks_total),
                 offsetof(pvf_spec, z_min_mm), offsetof(pvf_spec, integral_min), offsetof(pvf_spec, half_window),
                 offsetof(pvf_spec, boundary_mm), offsetof(pvf_spec, unet_layout));
          printf("%zu %zu %zu\\n", sizeof(pvf_tracks), offsetof(pvf_tracks, d_event_offsets),
                 offsetof(pvf_tracks, d_feat));
          printf("%zu %zu\\n", sizeof(pvf_vertices), offsetof(pvf_vertices, d_bin));
          return 0;
        }"""))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    a = [int(x) for x in lines[0].split()]
    assert a == [C.sizeof(B.Spec), B.Spec.max_tracks_total.offset, B.Spec.z_min_mm.offset,
                 B.Spec.integral_min.offset, B.Spec.half_window.offset, B.Spec.boundary_mm.offset,
                 B.Spec.unet_layout.offset]
    b = [int(x) for x in lines[1].split()]
    assert b == [C.sizeof(B.Tracks), B.Tracks.d_event_offsets.offset, B.Tracks.d_feat.offset]
    c = [int(x) for x in lines[2].split()]
    assert c == [C.sizeof(B.Vertices), B.Vertices.d_bin.offset]


def test_default_spec():
    s = pv.default_spec()
    assert (s.n_bins, s.bins_per_interval, s.n_levels, s.base_channels) == (4000, 100, 4, 32)
    assert s.z_min_mm == -100.0 and s.bin_width_mm == 0.1
    assert (s.peak_min, s.integral_min, s.half_window) == (0.01, 0.2, 5)
    assert s.compute_dtype == 0 and s.abi_version == 1
    assert s.boundary_mm == 0.0 and s.unet_layout == 0


def test_interval_layout_shapes():
    """One UNet sequence per interval: 100 bins need 3 levels (100/50/25);
    the arena grows by the extra guard rows of 40 sequences."""
    ok = pv.default_spec(max_events=1, unet_layout=1, n_levels=3)
    ev = pv.default_spec(max_events=1, n_levels=3)
    assert pv.arena_bytes(ok) > pv.arena_bytes(ev)
    bad = pv.default_spec(max_events=1, unet_layout=1, bins_per_interval=50)   # 50 % 8 != 0
    n = C.c_size_t(0)
    assert pv.load_library().pvf_arena_bytes(C.byref(bad), C.byref(n)) == 2


def test_arena_bytes_scales_with_events():
    a1 = pv.arena_bytes(pv.default_spec(max_events=1))
    a2 = pv.arena_bytes(pv.default_spec(max_events=101))
    per_event = (a2 - a1) / 100
    # activations: x0 + per level (a, cat, pool, d) in FP32, channels-last with guard rows
    assert 7.2e6 < per_event < 7.8e6
    assert a1 % 256 == 0


@pytest.mark.parametrize("field,value,status", [
    ("abi_version", 7, 1), ("max_events", 0, 1), ("max_peaks_per_event", 0, 1),
    ("max_tracks_total", -1, 1), ("compute_dtype", 9, 1),
    ("compute_dtype", -1, 1), ("n_levels", 1, 2), ("base_channels", 48, 2), ("n_bins", 4001, 2),
    ("bins_per_interval", 300, 2), ("bin_width_mm", 0.0, 1), ("half_window", -1, 1),
    ("max_peaks_per_event", 5000, 2), ("base_channels", 16, 2), ("base_channels", 64, 0),
    ("boundary_mm", -0.5, 1), ("boundary_mm", 5.01, 1), ("boundary_mm", 5.0, 0), ("boundary_mm", float("nan"), 1),
    ("unet_layout", 2, 1), ("unet_layout", 1, 2), ("reserved", 3, 1),
])
def test_spec_validation(field, value, status):
    s = pv.default_spec()
    setattr(s, field, value)
    n = C.c_size_t(0)
    assert pv.load_library().pvf_arena_bytes(C.byref(s), C.byref(n)) == status


def _init(spec, blob, arena=256, arena_bytes=None, stream=8):
    lib = pv.load_library()
    h = C.c_void_p(None)
    nb = arena_bytes if arena_bytes is not None else pv.arena_bytes(spec)
    st = lib.pvf_init(C.byref(spec), blob, len(blob), C.c_void_p(arena), nb, C.c_void_p(stream), C.byref(h))
    return st, h


def test_init_host_checks_before_device_work():
    """Each case fails validation before the library touches the device (the
    arena and stream given are never dereferenced)."""
    spec = pv.default_spec(max_events=4)
    good = weights_to_blob(make_weights(0))
    assert _init(spec, good, stream=0)[0] == 1                    # null stream
    assert _init(spec, good, arena=0)[0] == 1                     # null arena
    assert _init(spec, good, arena=258)[0] == 8                   # misaligned arena
    assert _init(spec, good, arena_bytes=pv.arena_bytes(spec) - 1)[0] == 4
    assert _init(spec, good[:-4])[0] == 5                         # truncated blob
    assert _init(spec, good + b"\0\0\0\0")[0] == 5                # trailing bytes
    assert _init(spec, b"XXXX" + good[4:])[0] == 5                # bad magic
    other = weights_to_blob(make_weights(0, shape=NetShape(n_levels=3)))
    assert _init(spec, other)[0] == 5                             # shape != spec
    w = make_weights(0)
    w.tensors["enc1.c1.w"] = w.tensors["enc1.c1.w"].copy()
    w.tensors["enc1.c1.w"][0, 0, 0] = float("nan")
    assert _init(spec, weights_to_blob(w))[0] == 5                # non-finite weight
    st, h = _init(spec, good, stream=0)
    assert h.value is None


def test_fp8_needs_calibration_table():
    """An FP8 engine is built only from a calibration table of the right size;
    pvf_init refuses the FP8 spec, pvf_init_fp8 refuses the other dtypes, and
    both answer before any device work."""
    lib = pv.load_library()
    spec = pv.default_spec(max_events=4, compute_dtype=3)
    blob = weights_to_blob(make_weights(0))
    n = C.c_size_t(0)
    assert lib.pvf_arena_bytes(C.byref(spec), C.byref(n)) == 0
    assert _init(spec, blob)[0] == 1
    h = C.c_void_p(None)
    amax = (C.c_float * 4)(1, 1, 1, 1)
    st = lib.pvf_init_fp8(C.byref(spec), blob, len(blob), None, 0, C.c_void_p(256), n.value, C.c_void_p(8),
                          C.byref(h))
    assert st == 1 and h.value is None
    st = lib.pvf_init_fp8(C.byref(pv.default_spec(max_events=4)), blob, len(blob), amax, 4, C.c_void_p(256),
                          n.value, C.c_void_p(8), C.byref(h))
    assert st == 1
    assert lib.pvf_calibration_size(None) == -1
    assert lib.pvf_calibrate(None, None, None, None, 0) == 1


def test_execute_rejects_null_engine():
    lib = pv.load_library()
    tr, v = B.Tracks(), B.Vertices()
    assert lib.pvf_execute(None, C.byref(tr), C.byref(v)) == 1
    assert lib.pvf_execute_scratch(None, C.byref(tr), C.byref(v)) == 1
    assert lib.pvf_destroy(None) == 1
    assert lib.pvf_launch_count(None) == 0


def test_status_strings():
    lib = pv.load_library()
    for k in range(10):
        assert lib.pvf_status_string(k) and lib.pvf_status_string(k) != b"unknown status"
    assert b"scratch" in lib.pvf_status_string(9)
    assert lib.pvf_status_string(99) == b"unknown status"


def test_scratch_size_in_header_matches_library_limit():
    """PVF_SCRATCH_BYTES (the header's stated limit of pvf_execute_scratch)
    is 64 MiB, and the status text names the same limit."""
    import re
    text = open(os.path.join(ROOT, "include", "pvf.h")).read()
    m = re.search(r"#define PVF_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == 64 << 20
    assert b"64 MiB" in pv.load_library().pvf_status_string(9)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(B, "_LIB", None)
    with pytest.raises(ImportError):
        B.load_library()
